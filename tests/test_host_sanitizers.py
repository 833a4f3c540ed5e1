"""The host-side mesh and sparse-Cholesky code (mesh_host.cpp, chol_host.cpp:
adjacency of Eq. 2, normal matrix of Eq. 12, nested dissection, symbolic and
numeric supernodal factorisation, host solve) built with g++'s address and
undefined-behaviour sanitizers and run on small meshes and on meshes it must
reject.  An out-of-bounds access, a use after free, a leak or undefined
arithmetic makes the driver (tests/native/host_check.cpp) report and fail.
CPU only."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from synth import animate, meshes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2111_10105_amd", "csrc")
DRIVER = os.path.join(ROOT, "tests", "native", "host_check.cpp")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("asan") / "host_check")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-fopenmp", "-o", exe,
           DRIVER, os.path.join(CSRC, "mesh_host.cpp"), os.path.join(CSRC, "chol_host.cpp")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "asan" in r.stderr.lower():
        pytest.skip("sanitizer runtime not available: " + r.stderr[-300:])
    assert r.returncode == 0, r.stderr[-2000:]
    return exe


def _run(driver, tmp_path, n, tris, anchors, lap=0, leaf=16):
    path = str(tmp_path / "mesh.bin")
    tris = np.asarray(tris, dtype=np.int32).reshape(-1, 3)
    anchors = np.asarray(anchors, dtype=np.int32)
    hdr = np.array([n, tris.shape[0], anchors.size, lap, leaf], dtype=np.int32)
    with open(path, "wb") as f:
        f.write(hdr.tobytes() + tris.tobytes() + anchors.tobytes())
    env = dict(os.environ, OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=99",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=98")
    r = subprocess.run([driver, path], capture_output=True, text=True, env=env, timeout=300)
    assert "Sanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-3000:]
    return r.returncode, r.stdout


@pytest.mark.parametrize("lap", [0, 1])
@pytest.mark.parametrize("mesh", ["torus", "icosphere"])
def test_factor_and_solve_clean(driver, tmp_path, mesh, lap):
    v, t = meshes.torus(14, 11) if mesh == "torus" else meshes.icosphere(3)
    n = v.shape[0]
    anchors = animate.choose_anchors(n, 5, seed=3)
    for leaf in (4, 16, 4096):  # many levels, a few, one supernode
        rc, out = _run(driver, tmp_path, n, t, anchors, lap, leaf)
        assert rc == 0, out
        resid = float(out.split("resid")[1])
        assert resid < 1e-10, out


def test_two_components_each_anchored(driver, tmp_path):
    v, t = meshes.torus(8, 6)
    n = v.shape[0]
    tris = np.concatenate([t, t + n])
    rc, out = _run(driver, tmp_path, 2 * n, tris, [0, n + 1])
    assert rc == 0, out


def test_rejected_meshes(driver, tmp_path):
    v, t = meshes.torus(8, 6)
    n = v.shape[0]
    bad = t.copy()
    bad[3, 1] = n  # index out of range
    rc, out = _run(driver, tmp_path, n, bad, [0])
    assert rc == 2 and "range" in out, out
    bad[3, 1] = -1
    rc, out = _run(driver, tmp_path, n, bad, [0])
    assert rc == 2, out
    tris = np.concatenate([t, t + n])  # second component without an anchor
    rc, out = _run(driver, tmp_path, 2 * n, tris, [0])
    assert rc == 3, out
