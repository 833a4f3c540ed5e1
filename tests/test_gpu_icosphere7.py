"""Parity at the precision form's size: icosphere level 7 (163,842 vertices),
windows of 64 frames, k = 32, 10-bit codes, 1,638 anchors, two chained
windows from a seeded Gaussian start, float32 frames, in the float32 form
and the precision form (bfloat16 covariance and C.Q).  This reaches the
T <= 64 / k <= 32 class of the orthogonal iterations, the 32-row
projection, the 12-level factor of the normal matrix and the direct decode
form (with this many anchors the mesh holds no anchor response).  The float64
oracle takes about a minute and a half here.  Needs an MI355X."""
import numpy as np
import pytest

import oracle as O
from paper_2111_10105_amd import dmc
from synth import animate, configs

from gpu_helpers import to_dev

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(1200)]

FRAMES, T, K, BITS = 128, 64, 32, 10
START_SEED = 909


@pytest.fixture(scope="module")
def case(gpu):
    w = configs.icosphere7(frames=FRAMES)
    q0 = animate.gaussian_subspace(T, K, START_SEED)
    recs, ref = O.compress_sequence(w.n, w.tris, w.frames, w.anchors, T, K, BITS,
                                    first_start=q0, fp32_data=True)
    ctx = dmc.Context(0)
    mesh = dmc.Mesh(ctx, w.n, w.tris, w.anchors)
    yield w, q0, recs, ref, ctx, mesh
    ctx.close()


def _np(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("prec", [dmc.FP32, dmc.BF16])
def test_codes_bit_exact_on_gpu_coefficients(case, prec):
    """Each window's coefficient codes and row ranges (Eq. 10) equal the
    oracle quantiser's on the coefficients the GPU computed, and the anchor
    codes the oracle's on the same frames, bit for bit."""
    w, q0, _, _, ctx, mesh = case
    p = dmc.make_params(K, coef_bits=BITS, precision=prec)
    start = to_dev(q0.astype(np.float32))
    for wi in range(FRAMES // T):
        fr = w.frames[wi * T:(wi + 1) * T]
        r = dmc.encode_window(ctx, mesh, to_dev(fr), p, q_start=start, want_coef=True)
        assert r["status"] == 0, r["stats"]
        view = dmc.parse_record(_np(r["code"]), w.n, T, mesh.nc, p)
        coef = _np(r["coef"])
        for c in range(3):
            codes, ranges, _ = O.quantise_rows(coef[c].astype(np.float64), BITS, fp32_data=True)
            assert np.array_equal(view.ranges[c], ranges)
            assert np.array_equal(view.codes[c], codes)
            a = O.anchor_values(fr, w.anchors, c)
            lo, hi = O.stored_range(a.astype(np.float32))
            assert np.array_equal(view.anchor_range[c], np.array([lo, hi], dtype=np.float32))
            assert np.array_equal(view.anchor_codes[c], O.quantise_uniform(a, lo, hi, 16).T)
        start = r["u"]


def test_float32_form_against_oracle(case):
    """The float32 form's reconstruction of the two chained windows is within
    NMSE 1e-5 of the oracle's, its error against the input within 10% of the
    oracle's, and its subspaces within the angle the float32 data allows."""
    w, q0, recs, ref, ctx, mesh = case
    p = dmc.make_params(K, coef_bits=BITS, precision=dmc.FP32)
    codes, out, stats, status = dmc.compress_sequence(ctx, mesh, to_dev(w.frames), T, p,
                                                      q_start=to_dev(q0.astype(np.float32)))
    assert status == 0, stats
    got = _np(out)
    e_or, e_in, r_in = O.nmse(got, ref), O.nmse(got, w.frames), O.nmse(ref, w.frames)
    print(f"fp32: NMSE(gpu,oracle)={e_or:.3e} NMSE(gpu,input)={e_in:.6e} "
          f"NMSE(oracle,input)={r_in:.6e} sweeps={[s['oi_sweeps'] for s in stats]} "
          f"cg={stats[0]['cg_iters']} {stats[0]['cg_resid']:.2e}")
    assert e_or <= 1e-5
    assert e_in <= 1.1 * r_in
    assert not dmc.Mesh.anchor_response(mesh)[0]  # the direct decode form ran


def test_precision_form_against_oracle(case):
    """The precision form at the same size: NMSE against the oracle within
    1e-5, and its sweeps stated beside the float32 form's."""
    w, q0, _, ref, ctx, mesh = case
    p = dmc.make_params(K, coef_bits=BITS, precision=dmc.BF16)
    codes, out, stats, status = dmc.compress_sequence(ctx, mesh, to_dev(w.frames), T, p,
                                                      q_start=to_dev(q0.astype(np.float32)))
    got = _np(out)
    e_or, e_in, r_in = O.nmse(got, ref), O.nmse(got, w.frames), O.nmse(ref, w.frames)
    print(f"bf16: status={status} NMSE(gpu,oracle)={e_or:.3e} NMSE(gpu,input)={e_in:.6e} "
          f"NMSE(oracle,input)={r_in:.6e} sweeps={[s['oi_sweeps'] for s in stats]} "
          f"resid={[s['oi_resid'] for s in stats]}")
    assert status in (0, 4)
    assert e_or <= 1e-5
    assert e_in <= 1.1 * r_in
