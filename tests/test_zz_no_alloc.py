"""The encode entry point that allocates nothing (its scratch is a fixed
device array of the library): through the C ABI, two calls in a row, the
second with a smaller window, each against dmc_encode_window on the same
inputs; and a window beyond the array's size is refused.  Needs an MI355X."""
import ctypes

import numpy as np
import pytest

from paper_2111_10105_amd import dmc
from synth import animate, configs, meshes

from gpu_helpers import to_dev

pytestmark = pytest.mark.gpu

BUFFER_TOO_SMALL = 6


def _encode(ctx, mesh, frames, p, q0, noalloc):
    import torch
    T = frames.shape[0]
    k = min(p.k, T)
    code = torch.full((dmc.window_code_bytes(mesh.n, T, mesh.nc, p),), 0xAB, dtype=torch.uint8,
                      device=frames.device)
    u = torch.empty((3, T, k), dtype=frames.dtype, device=frames.device)
    coef = torch.empty((3, k, mesh.n), dtype=frames.dtype, device=frames.device)
    st = dmc.WindowStats()
    ctx.sync_stream()
    fn = dmc.lib().dmc_encode_window_noalloc if noalloc else dmc.lib().dmc_encode_window
    status = fn(ctx.h, mesh.h, dmc._ptr(frames), T, ctypes.byref(p), dmc._ptr(q0), dmc._ptr(code),
                dmc._ptr(u), dmc._ptr(coef), ctypes.byref(st))
    torch.cuda.synchronize()
    return status, code.cpu().numpy(), u.cpu().numpy(), coef.cpu().numpy(), st.as_dict()


@pytest.mark.parametrize("prec", [dmc.FP32, dmc.FP64])
def test_noalloc_encode_matches_encode_window(gpu, prec):
    dt = np.float64 if prec == dmc.FP64 else np.float32
    ctx = dmc.Context(0)
    try:
        big = configs.torus_fp32(frames=32)  # 16,384 vertices, T = 32, k = 16
        v, t = meshes.icosphere(3)           # 642 vertices, T = 24, k = 4
        small_frames = animate.bend_twist(v, 24, seed=3, noise_var=1e-6, dtype=dt)
        cases = [(big.n, big.tris, big.anchors, big.frames.astype(dt), big.k),
                 (v.shape[0], t, animate.choose_anchors(v.shape[0], 6, 1), small_frames, 4)]
        for n, tris, anchors, fr, k in cases:
            mesh = dmc.Mesh(ctx, n, tris, anchors)
            T = fr.shape[0]
            p = dmc.make_params(k, coef_bits=12, precision=prec)
            q0 = to_dev(animate.gaussian_subspace(T, k, 11).astype(dt))
            frames = to_dev(fr)
            ref = _encode(ctx, mesh, frames, p, q0, noalloc=False)
            got = _encode(ctx, mesh, frames, p, q0, noalloc=True)
            print(f"n={n} T={T} k={k}: status {ref[0]} / {got[0]}, sweeps {ref[4]['oi_sweeps']}")
            assert ref[0] == 0 and got[0] == 0, (ref[0], got[0], dmc.lib().dmc_last_error())
            for a, b in zip(ref[1:4], got[1:4]):
                assert np.array_equal(a, b)
            assert got[4]["oi_sweeps"] == ref[4]["oi_sweeps"]
            assert got[4]["q_s"] == ref[4]["q_s"]
    finally:
        ctx.close()


def test_noalloc_refuses_windows_beyond_its_array(gpu):
    import torch
    ctx = dmc.Context(0)
    try:
        w = configs.icosphere7(frames=64)  # 163,842 vertices x 64 frames: above the limit
        mesh = dmc.Mesh(ctx, w.n, w.tris, w.anchors)
        p = dmc.make_params(w.k, coef_bits=w.bits, precision=dmc.FP32)
        # its frames alone (125.8 MB of delta coordinates) exceed the array
        assert w.T * w.n * 3 * 4 > dmc.NOALLOC_SCRATCH_BYTES
        frames = to_dev(w.frames)
        code = torch.empty(dmc.window_code_bytes(w.n, w.T, mesh.nc, p), dtype=torch.uint8,
                           device="cuda:0")
        ctx.sync_stream()
        status = dmc.lib().dmc_encode_window_noalloc(ctx.h, mesh.h, dmc._ptr(frames), w.T,
                                                     ctypes.byref(p), None, dmc._ptr(code), None,
                                                     None, None)
        assert status == BUFFER_TOO_SMALL
        assert b"fixed array" in dmc.lib().dmc_last_error()
    finally:
        ctx.close()
