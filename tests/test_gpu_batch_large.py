"""The largest sequences of the 64-sequence batched workload (tori and
icospheres of 2k-60k vertices, 16-128 frames, k in {8, 16, 32}, T = 2k,
seed 4000), drawn exactly as in the full batch and run through one batch
graph as the benchmark runs it (exact start per window, one conjugate-
gradient iteration with the Cholesky preconditioner), against the float64
oracle.  Needs an MI355X."""
import numpy as np
import pytest

import oracle as O
from paper_2111_10105_amd import dmc
from synth import configs

from gpu_helpers import to_dev

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

# the three largest by vertex-frames (torus 225x225 x 114 frames, k = 8;
# torus 216x215 x 108, k = 16) and the largest icosphere with k = 16
# (level 6 x 111 frames)
LARGEST = (24, 59, 28)


def _np(t):
    return t.detach().cpu().numpy()


def test_largest_batched_sequences_against_oracle(gpu):
    ws = configs.batched(only=LARGEST)
    assert len(ws) == len(LARGEST)
    ctx = dmc.Context(0)
    try:
        meshes = [dmc.Mesh(ctx, w.n, w.tris, w.anchors) for w in ws]
        frames = [to_dev(w.frames) for w in ws]
        params = [dmc.make_params(w.k, coef_bits=w.bits, precision=dmc.FP32, init=dmc.INIT_EXACT,
                                  cg_max_iters=1) for w in ws]
        b = dmc.Batch(ctx, meshes, frames, [w.T for w in ws], params)
        try:
            b.run()
            for i, w in enumerate(ws):
                stats, status = b.stats(i)
                assert status == 0, stats
                got = _np(b.out[i])
                _, ref = O.compress_sequence(w.n, w.tris, w.frames, w.anchors, w.T, w.k, w.bits,
                                             init="exact", fp32_data=True)
                e_or, e_in, r_in = O.nmse(got, ref), O.nmse(got, w.frames), O.nmse(ref, w.frames)
                print(f"{w.name} ({w.n} vertices): NMSE(batch,oracle)={e_or:.3e} "
                      f"NMSE(batch,input)={e_in:.6e} NMSE(oracle,input)={r_in:.6e}")
                assert e_or <= 1e-5
                # RBF motion: the trailing eigenvalues of these windows lie at
                # round-off, where the discarded directions are not fixed by
                # the data, so the error against the input is held to 10% of
                # the oracle's
                assert e_in <= 1.1 * r_in
        finally:
            b.close()
    finally:
        ctx.close()
