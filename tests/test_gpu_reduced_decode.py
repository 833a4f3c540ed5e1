"""The temporal-subspace decode (include/dmc.h, dmc_mesh_anchor_response):
the right-hand side of Eq. (12) is linear in the decoded delta coordinates and
anchor values, so the decoder solves the 3k columns L^T Y^^T of each window and
forms X = Z U~^T + G A^ with the mesh's anchor response G.  Checked against
the defining property: every decoded frame satisfies its full normal
equations (L^T L + I_N^T I_N) X_t = L^T Delta~_t + I_N^T A^_t to the
conjugate-gradient tolerance, with Delta~ and A^ rebuilt on the host by the
oracle's dequantiser from the records."""
import numpy as np
import pytest

import oracle as O
from paper_2111_10105_amd import dmc
from synth import configs

from gpu_helpers import record_to_oracle, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(gpu):
    c = dmc.Context(0)
    yield c
    c.close()


def _np(t):
    return t.detach().cpu().numpy()


def test_anchor_response_built(ctx):
    w = configs.small_torus()
    m = dmc.Mesh(ctx, w.n, w.tris, w.anchors)
    built, iters, resid = m.anchor_response()
    assert built and iters >= 1 and resid <= 1e-12, (built, iters, resid)


def _full_residuals(w, lap, p, codes, out):
    """Relative residual of every frame's (and coordinate's) full normal
    equations, in float64 on the host."""
    L = O.laplacian(w.n, w.tris, O.LAP_UNIFORM if lap == dmc.LAP_UNIFORM else O.LAP_COMBINATORIAL)
    A = O.normal_matrix(L, w.anchors)
    P = O.selection(w.n, w.anchors)
    buf = _np(codes)
    res = []
    off, t0 = 0, 0
    for T_w in [w.T] * (w.F // w.T) + ([w.F % w.T] if w.F % w.T else []):
        nb = dmc.window_code_bytes(w.n, T_w, w.anchors.size, p)
        rec = record_to_oracle(dmc.parse_record(buf[off:off + nb], w.n, T_w, w.anchors.size, p),
                               p, T_w)
        for c in range(3):
            delta = rec["Y_hat"][c].T @ rec["U_tilde"][c].T      # n x T_w
            B = L.T @ delta + P.T @ rec["A_hat"][c]              # n x T_w
            X = out[t0:t0 + T_w, :, c].T.astype(np.float64)      # n x T_w
            R = A @ X - B
            res.append(np.linalg.norm(R, axis=0) / np.linalg.norm(B, axis=0))
        off += nb
        t0 += T_w
    return np.concatenate(res)


@pytest.mark.parametrize("lap", [dmc.LAP_UNIFORM, dmc.LAP_COMBINATORIAL])
@pytest.mark.parametrize("precond", [dmc.PRECOND_NONE, dmc.PRECOND_JACOBI,
                                     dmc.PRECOND_CHOLESKY])
@pytest.mark.parametrize("tol", [1e-6, 1e-9])
def test_every_frame_meets_the_tolerance(ctx, lap, precond, tol):
    """40 frames in windows of 16 (a short tail), k = 6 < T: the reduced
    columns' convergence test bounds each frame's full relative residual.
    (Tolerances well above the floor where the recursively updated CG
    residual parts from the true one.)"""
    w = configs.small_torus(frames=40, T=16, k=6)
    m = dmc.Mesh(ctx, w.n, w.tris, w.anchors, lap)
    assert m.anchor_response()[0]
    p = dmc.make_params(w.k, coef_bits=w.bits, precision=dmc.FP64, cg_tol=tol, precond=precond,
                        cg_max_iters=2000)
    codes, _, _, _ = dmc.compress_sequence(ctx, m, to_dev(w.frames), w.T, p, decode=False)
    out, st, status = dmc.decode_sequence(ctx, m, codes, w.F, w.T, p)
    assert status == 0, st
    res = _full_residuals(w, lap, p, codes, _np(out))
    assert res.max() <= 1.01 * tol, (res.max(), st[0])
