"""Run-to-run reproducibility of the GPU path on the benchmark workload
(torus 128 x 128, 256 frames in windows of 32, k = 16, 12-bit codes, 64
anchors, float32): every reduction in the library adds its terms in a fixed
order (wavefront sums by fixed lane pairings, split-K partial tiles of the
backward solve in split order), so two runs on the same input give the same
bits.  Checked for the codes, the decoded frames and the decode of stored
codes alone."""
import numpy as np
import pytest
import torch

from paper_2111_10105_amd import dmc
from synth import animate, configs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(gpu):
    c = dmc.Context(0)
    yield c
    c.close()


def test_same_bits_twice(ctx):
    w = configs.torus_fp32()
    dev = torch.device("cuda:0")
    frames = torch.from_numpy(w.frames).to(dev)
    q0 = torch.from_numpy(animate.gaussian_subspace(w.T, w.k, 12345).astype(np.float32)).to(dev)
    mesh = dmc.Mesh(ctx, w.n, w.tris, w.anchors)
    p = dmc.make_params(w.k, coef_bits=w.bits, precision=dmc.FP32)
    nbytes = dmc.sequence_code_bytes(w.n, w.F, w.T, mesh.nc, p)
    runs = []
    for _ in range(2):
        codes = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        out = torch.empty_like(frames)
        _, _, _, status = dmc.compress_sequence(ctx, mesh, frames, w.T, p, q_start=q0,
                                                codes=codes, out=out, stats=True)
        assert status == 0
        torch.cuda.synchronize()
        runs.append((codes.cpu().numpy(), out.cpu().numpy()))
    assert np.array_equal(runs[0][0], runs[1][0])
    assert np.array_equal(runs[0][1].view(np.uint32), runs[1][1].view(np.uint32))
    # decoding the stored codes again gives the same frames
    again = torch.empty_like(frames)
    dmc.decode_sequence(ctx, mesh, torch.from_numpy(runs[0][0]).to(dev), w.F, w.T, p, out=again)
    torch.cuda.synchronize()
    assert np.array_equal(again.cpu().numpy().view(np.uint32), runs[0][1].view(np.uint32))
