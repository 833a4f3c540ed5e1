"""The normal matrix's sparse Cholesky factor computed on the device at mesh
creation (numeric supernodal factorisation level by level from the host's
ordering and symbolic analysis, then the solve operators): one forward and
one backward solve with it (dmc_mesh_normal_solve) reproduce SciPy's sparse
LU solution of (L^T L + I_N^T I_N) X = B (Eq. 12's normal equations) to 1e-9
relative, on meshes with one and many tree levels, a boundary, two
components and both Laplacians, and up to the headline mesh.  Needs an
MI355X."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle as O
from paper_2111_10105_amd import dmc
from synth import animate, meshes

from gpu_helpers import to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(gpu):
    c = dmc.Context(0)
    yield c
    c.close()


def _case(name):
    if name == "torus":
        v, t = meshes.torus(30, 24)
    elif name == "grid":
        v, t = meshes.grid(40, 33)
    elif name == "two_tori":
        v, t = meshes.torus(12, 10)
        t = np.concatenate([t, t + v.shape[0]])
        v = np.concatenate([v, v + 3.0])
    elif name == "ico5":
        v, t = meshes.icosphere(5)
    elif name == "tiny":
        v, t = meshes.icosphere(1)
    return v, t


@pytest.mark.parametrize("lap", [dmc.LAP_UNIFORM, dmc.LAP_COMBINATORIAL])
@pytest.mark.parametrize("name", ["tiny", "torus", "grid", "two_tori", "ico5"])
def test_device_factor_solves_normal_equations(ctx, name, lap):
    v, t = _case(name)
    n = v.shape[0]
    if name == "two_tori":
        anchors = np.array([0, 5, n // 2 + 3], dtype=np.int32)
    else:
        anchors = animate.choose_anchors(n, max(3, n // 100), seed=11)
    m = dmc.Mesh(ctx, n, t, anchors, laplacian=lap)
    kind = "uniform" if lap == dmc.LAP_UNIFORM else "combinatorial"
    M = O.normal_matrix(O.laplacian(n, t, kind), anchors).tocsc()
    rng = np.random.default_rng(5)
    B = rng.standard_normal((n, 7))
    X = dmc.normal_solve(ctx, m, to_dev(B)).cpu().numpy()
    ref = spla.splu(M).solve(B)
    rel = np.max(np.abs(X - ref)) / np.max(np.abs(ref))
    res = np.max(np.abs(M @ X - B)) / np.max(np.abs(B))
    info = m.factor_info()
    print(f"{name} lap {lap}: n {n} levels {info['levels']:.0f} supernodes "
          f"{info['supernodes']:.0f} rel {rel:.2e} residual {res:.2e} {info['seconds']:.3f} s")
    assert rel < 1e-9 and res < 1e-9


def test_device_factor_headline_mesh(ctx):
    """Icosphere level 7 with 1% anchors (12 tree levels, blocks up to 2,029
    rows): the device factor against SciPy, and its setup time."""
    v, t = meshes.icosphere(7)
    n = v.shape[0]
    anchors = animate.choose_anchors(n, n // 100, seed=3)
    m = dmc.Mesh(ctx, n, t, anchors)
    info = m.factor_info()
    M = O.normal_matrix(O.laplacian(n, t), anchors).tocsc()
    B = np.random.default_rng(9).standard_normal((n, 3))
    X = dmc.normal_solve(ctx, m, to_dev(B)).cpu().numpy()
    ref = spla.splu(M).solve(B)
    rel = np.max(np.abs(X - ref)) / np.max(np.abs(ref))
    print(f"icosphere 7: rel {rel:.2e}, factor built in {info['seconds']:.3f} s")
    assert rel < 1e-9


def test_normal_solve_rejects_bad_arguments(ctx):
    import torch
    v, t = meshes.icosphere(2)
    m = dmc.Mesh(ctx, v.shape[0], t, np.array([0, 7], dtype=np.int32))
    B = torch.zeros((v.shape[0], 2), dtype=torch.float64, device="cuda:0")
    st = dmc.lib().dmc_mesh_normal_solve(ctx.h, m.h, 0, dmc._ptr(B), dmc._ptr(B))
    assert st == 1  # ncols < 1
    st = dmc.lib().dmc_mesh_normal_solve(ctx.h, m.h, 2, dmc._ptr(B), dmc._ptr(B))
    assert st == 1  # aliasing
