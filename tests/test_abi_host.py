"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every symbol declared in include/dmc.h, and its pure host functions (record
sizes) agree with the documented layout."""
import ctypes
import os
import re

import pytest

from paper_2111_10105_amd import dmc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "dmc.h")).read()
    return sorted(set(re.findall(r"\b(dmc_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = dmc.lib()
    names = _declared()
    assert "dmc_encode_window" in names and "dmc_compress_sequence" in names
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(dmc.EXPORTS)


def _align(x):
    return (x + 255) // 256 * 256


@pytest.mark.parametrize("prec,cb,ab,db", [(dmc.FP32, 12, 16, 16), (dmc.FP64, 0, 0, 0),
                                           (dmc.FP32, 10, 0, 16)])
def test_record_size_matches_layout(prec, cb, ab, db):
    p = dmc.make_params(16, coef_bits=cb, anchor_bits=ab, dict_bits=db, precision=prec)
    n, T, nc = 1000, 32, 10
    real = 8 if prec == dmc.FP64 else 4
    k = 16

    def words(count, bits):  # 32-bit words of a segment, even count; raw values if bits == 0
        w = (count * bits + 31) // 32 if bits else (count * real + 3) // 4
        return w + w % 2

    # header 128 B, column and row tables (16 B entries), anchor ranges; the
    # anchor segments; then the dictionary columns and the rows at their widest
    fixed = _align(128 + 2 * 3 * k * 16 + 24)
    anchors = _align(fixed + 3 * 4 * words(T * nc, ab))
    expect = _align(anchors + 4 * 3 * k * (words(T, db) + words(n, cb)))
    assert dmc.window_code_bytes(n, T, nc, p) == expect
    # a short window keeps k_w = min(k, T_w)
    assert dmc.window_code_bytes(n, 5, nc, p) < expect
    # sequence = full windows + tail
    assert dmc.sequence_code_bytes(n, 70, T, nc, p) == 2 * expect + dmc.window_code_bytes(n, 6, nc, p)


def test_invalid_arguments_report_errors_without_gpu():
    L = dmc.lib()
    # NULL context pointers are rejected on the host before any device call
    st = L.dmc_set_stream(None, None)
    assert st == 1 and b"NULL" in L.dmc_last_error()
    assert dmc.window_code_bytes(0, 32, 1, dmc.make_params(4)) == 0
    h = ctypes.c_void_p()
    st = L.dmc_mesh_create(None, 3, 1, None, 0, None, 0, ctypes.byref(h))
    assert st == 1


# ---------------------------------------------------------------- host factorisation

import numpy as np  # noqa: E402

import oracle as O  # noqa: E402
from synth import animate, meshes  # noqa: E402


@pytest.mark.parametrize("mesh,nc,lap", [
    ("torus", 6, dmc.LAP_UNIFORM), ("torus", 6, dmc.LAP_COMBINATORIAL),
    ("grid", 3, dmc.LAP_UNIFORM), ("ico3", 8, dmc.LAP_UNIFORM),
    ("two_parts", 4, dmc.LAP_UNIFORM), ("tiny", 1, dmc.LAP_UNIFORM)])
def test_host_factor_solve_matches_direct_solve(mesh, nc, lap):
    """The library's nested-dissection supernodal factor solves the normal
    equations of Eq. (12) to round-off (compared with SciPy's sparse LU on the
    oracle's normal matrix)."""
    v, t = {"torus": lambda: meshes.torus(30, 22), "grid": lambda: meshes.grid(25, 19),
            "ico3": lambda: meshes.icosphere(3),
            "two_parts": lambda: meshes.disjoint_union(meshes.icosphere(2), meshes.torus(12, 9)),
            "tiny": lambda: meshes.icosphere(0)}[mesh]()
    n = v.shape[0]
    if mesh == "two_parts":
        anchors = np.array([0, 5, 162, 200], dtype=np.int32)
    else:
        anchors = animate.choose_anchors(n, nc, seed=3)
    kind = O.LAP_UNIFORM if lap == dmc.LAP_UNIFORM else O.LAP_COMBINATORIAL
    L = O.laplacian(n, t, kind)
    M = O.normal_matrix(L, anchors)
    rng = np.random.default_rng(1)
    B = rng.standard_normal((n, 7))
    X, info = dmc.host_normal_solve(n, t, anchors, B, lap)
    import scipy.sparse.linalg as spla
    ref = spla.splu(M).solve(B)
    rel = np.max(np.abs(X - ref)) / np.max(np.abs(ref))
    assert rel < 1e-9, rel
    assert np.max(np.abs(M @ X - B)) / np.max(np.abs(B)) < 1e-9
    assert info["stored"] >= info["nnz_exact"] - n  # every factor entry is stored
    assert info["levels"] >= 1 and info["supernodes"] >= 1
    # the leaves' columns: some, and all of them when the tree is one level
    assert 0 < info["leaf_rows"] <= n
    assert (info["leaf_rows"] == n) == (info["levels"] == 1)


def test_host_factor_rejects_unanchored_component():
    v, t = meshes.disjoint_union(meshes.icosphere(1), meshes.icosphere(1))
    with pytest.raises(dmc.DmcError) as e:
        dmc.host_normal_solve(v.shape[0], t, np.array([0, 1]), np.ones((v.shape[0], 1)))
    assert e.value.status == 5
