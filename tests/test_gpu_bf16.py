"""The precision form (bfloat16 covariance and C.Q products with float32
accumulation, full-precision refinement sweep, float64 Cholesky and Ritz)
through the C ABI: its covariance against the float64 oracle on the
bfloat16-rounded frames, and its reconstruction error against the float64
oracle's, stated per case."""
import numpy as np
import pytest

import oracle as O
from oracle import mlp_oracle as M
from paper_2111_10105_amd import dmc
from synth import animate, configs, meshes

from gpu_helpers import sin_angle, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(gpu):
    c = dmc.Context(0)
    yield c
    c.close()


def _np(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("T", [1, 7, 32, 40, 64])
def test_bf16_autocorrelation_matches_oracle_on_rounded_frames(ctx, T):
    """Products of bfloat16 values are exact in float32; only the float32
    accumulation over each vertex block rounds (the blocks are added in
    float64), so R matches the oracle's R of the bfloat16-rounded frames to
    ~1e-6 relative."""
    v, t = meshes.torus(25, 41)  # n = 1025: ragged against the 64-vertex tiles
    n = v.shape[0]
    fr = animate.rbf_skinning(v, T, 5, seed=T, dtype=np.float32)
    m = dmc.Mesh(ctx, n, t, animate.choose_anchors(n, 3, 1))
    R = _np(dmc.autocorrelation(ctx, m, to_dev(fr), dmc.BF16))
    frb = M.bf16_round(fr).reshape(fr.shape)
    for c in range(3):
        ref = O.autocorrelation(O.coordinate_matrix(frb, c))
        err = np.max(np.abs(R[c] - ref)) / np.abs(ref).max()
        assert err <= 2e-6, (c, err)


def test_bf16_window_subspace_close_to_fp32(ctx):
    """One window: the bfloat16 form's dominant eigen-trajectories match the
    float64 oracle's within the perturbation bfloat16 rounding of the frames
    implies (relative 2^-9 per value), on gapped directions."""
    T, k = 32, 4
    v, t = meshes.icosphere(3)
    fr = animate.bend_twist(v, T, seed=13, noise_var=1e-6, dtype=np.float32)
    anchors = animate.choose_anchors(v.shape[0], 7, seed=13)
    m = dmc.Mesh(ctx, v.shape[0], t, anchors)
    q0 = animate.gaussian_subspace(T, k, seed=7).astype(np.float32)
    p = dmc.make_params(k, precision=dmc.BF16, oi_tol=1e-12)
    r = dmc.encode_window(ctx, m, to_dev(fr), p, q_start=to_dev(q0))
    U = _np(r["u"]).astype(np.float64)
    st = r["stats"]
    for c in range(3):
        lam, V = O.jacobi_eigh(O.autocorrelation(O.coordinate_matrix(fr, c)))
        assert lam[k - 1] / lam[k] >= 10
        ang = sin_angle(V[:, :k], U[c])
        print(f"c{c}: sweeps {st['oi_sweeps'][c]} resid {st['oi_resid'][c]:.2e} angle {ang:.2e}")
        assert ang < 2e-2
        assert st["oi_sweeps"][c] >= 2  # bfloat16 stage + refinement


@pytest.mark.parametrize("init", [dmc.INIT_PREV, dmc.INIT_SKETCH])
def test_bf16_sequence_error_against_oracle(ctx, init):
    """The precision form on the small torus: its distance to the float64
    oracle's reconstruction is stated and bounded by the error of storing the
    frames in bfloat16."""
    w = configs.small_torus(frames=56, T=16, k=10, precision="fp32")
    m = dmc.Mesh(ctx, w.n, w.tris, w.anchors)
    p = dmc.make_params(w.k, coef_bits=w.bits, precision=dmc.BF16, cg_tol=1e-13, init=init)
    om = animate.gaussian_subspace(w.T, w.k, seed=80)[0].astype(np.float32)
    q = None if init == dmc.INIT_PREV else to_dev(om)
    codes, out, stats, status = dmc.compress_sequence(ctx, m, to_dev(w.frames), w.T, p, q_start=q)
    assert status == 0
    _, ref = O.compress_sequence(w.n, w.tris, w.frames, w.anchors, w.T, w.k, w.bits,
                                 init="prev" if init == dmc.INIT_PREV else "sketch",
                                 omega=om.astype(np.float64), fp32_data=True)
    got = _np(out)
    e_or, e_in, r_in = O.nmse(got, ref), O.nmse(got, w.frames), O.nmse(ref, w.frames)
    print(f"bf16 init {init}: sweeps {[s['oi_sweeps'] for s in stats]} NMSE(gpu,oracle)={e_or:.3e} "
          f"NMSE(gpu,input)={e_in:.3e} NMSE(oracle,input)={r_in:.3e}")
    # bar: the precision form's reconstruction is closer to the oracle's than
    # merely storing the input frames in bfloat16 would be
    e_store = O.nmse(M.bf16_round(w.frames).reshape(w.frames.shape), w.frames)
    print(f"  NMSE(bf16(frames), frames)={e_store:.3e}")
    assert e_or <= e_store
    assert all(s["oi_sweeps"] == [0, 0, 0] or min(s["oi_sweeps"]) >= 2 for s in stats)
