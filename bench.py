"""Benchmark: vertex-frames per second of encode + decode on one MI355X.

One step = the whole path over one synthetic sequence already resident in
HBM: delta coordinates, autocorrelation, orthogonal iterations with the Ritz
step, projection + quantisation, anchors (encode), then back-projection and the
anchored least-squares solve by preconditioned conjugate gradients on the
normal equations, and the transpose back to frames (decode).

Workload: 128 x 128 torus (16,384 vertices), 256 frames in windows of 32,
6-bone Gaussian-RBF skinning, k = 16, 12-bit codes, 64 anchors, float32 frames.
The first window's orthogonal iterations start from a seeded Gaussian block,
every later window from the previous window's subspace (Algorithm 1).

Prints one JSON line.  Besides the required keys it carries the per-family
kernel breakdown (HIP events per launch, outside the timed region) and the
roofline of the dominant family, timed live over the timed region.

`--gpus N` with N > 1 exits: this program measures one GPU.
`--copy-calibration MB` only runs a plain device-to-device copy of MB
megabytes (five times) and exits: the reference reading for the HBM byte
counters of the dominant kernel.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E, GB/s
FP64_PEAK_TFLOPS = 78.6    # MI355X FP64 matrix / vector, TFLOP/s
FIRST_START_SEED = 909     # seeded Gaussian start block of window 0

# source file of each kernel family (the byte counters of a family are valid
# only while its source is unchanged)
FAMILY_SOURCE = {
    "delta": "kernels_encode.hip", "autocorr": "kernels_encode.hip", "oi": "oi_device.h",
    "project": "kernels_encode.hip", "quantise": "kernels_encode.hip",
    "anchors": "kernels_encode.hip", "back_project": "kernels_decode.hip",
    "rhs": "kernels_decode.hip", "cg_spmm": "kernels_decode.hip",
    "cg_update": "kernels_decode.hip", "chol_fwd_gather": "kernels_chol.hip",
    "chol_fwd_solve": "kernels_chol.hip", "chol_bwd_solve": "kernels_chol.hip",
    "to_frames": "kernels_decode.hip",
}
FAMILY_KERNEL = {"chol_bwd_solve": "k_bwd_gemm", "chol_fwd_solve": "k_fwd_gemm",
                 "chol_fwd_gather": "k_fwd_gather", "oi": "k_oi", "cg_spmm": "k_cg_spmm",
                 "delta": "k_delta", "back_project": "k_back_project"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-kernel", default=None,
                    help="kernel family timed live (default: the dominant one)")
    ap.add_argument("--copy-calibration", type=float, default=0.0, metavar="MB")
    ap.add_argument("--workload", default="torus", choices=["torus", "icosphere7", "batched"],
                    help="torus: the headline workload; icosphere7: the precision form's "
                         "size; batched: 64 sequences in one graph")
    return ap.parse_args()


def source_hash(family: str) -> str:
    path = os.path.join(ROOT, "paper_2111_10105_amd", "csrc", FAMILY_SOURCE[family])
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(family: str):
    """HBM bytes per launch of `family` from the committed counter summary
    (profiles/<kernel>_torus128_pmc.txt), or None when there is none or the
    kernel source changed since the counters were taken."""
    kern = FAMILY_KERNEL.get(family)
    if kern is None:
        return None
    path = os.path.join(ROOT, "profiles", f"{kern}_torus128_pmc.txt")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_hash = re.search(r"^source_sha256_16:\s*(\S+)", text, re.M)
    m_bytes = re.search(r"^hbm_bytes_per_launch:\s*(\S+)", text, re.M)
    if not m_hash or not m_bytes or m_hash.group(1) != source_hash(family):
        return None
    return float(m_bytes.group(1))


def work_model(fam, *, n, F, T, k, nw, rs, ncols, nnz, m_nnz, finfo, sweeps_total, reduced=False,
               nc=0):
    """Algorithmic work of one step for a kernel family: (bound, amount, unit)
    with amount in bytes (hbm) or flops (mfma).  Bytes count each input read
    once and each output written once; flops count 2 per multiply-add of the
    operation's definition.  ncols: columns of the decoder's solve (3k per
    window with the mesh's anchor response, `reduced`, else 3F); nc anchors."""
    vec = 8.0 * n * ncols                     # one float64 n x ncols block
    fr = float(rs) * 3 * n * F                # the frames (or deltas) in their type
    coef = 3.0 * k * n * nw
    if fam == "delta":
        return "hbm", 2 * fr + 4.0 * (nnz + n + 1), "B"
    if fam == "autocorr":
        return "hbm", fr, "B"
    if fam == "oi":
        per = 2.0 * T * T * k + 2.0 * T * k * k + k ** 3 / 3.0
        return "mfma", per * sweeps_total, "flop"
    if fam == "project":
        return "hbm", fr + rs * coef, "B"
    if fam == "quantise":
        return "hbm", rs * coef + 2.0 * coef, "B"
    if fam == "back_project":  # reduced: the dequantised coefficient rows
        return "hbm", 2.0 * coef + vec, "B"
    if fam == "rhs":
        return "hbm", 2 * vec, "B"
    if fam == "cg_spmm":
        return "hbm", 2 * vec + 12.0 * m_nnz, "B"
    if fam == "cg_update":
        return "hbm", 6 * vec, "B"
    if fam == "chol_fwd_gather":
        return "hbm", 2 * vec + 8.0 * finfo["update_rows"] * ncols, "B"
    if fam in ("chol_fwd_solve", "chol_bwd_solve"):
        return "mfma", 2.0 * finfo["solve_entries"] * ncols, "flop"
    if fam == "to_frames":
        if reduced:  # X = Z U~^T + G A^ per window and coordinate, written as frames
            return "mfma", 2.0 * n * 3 * F * (nc + k), "flop"
        return "hbm", vec + fr, "B"
    return None, None, None


def train_learned_start(ctx, dmc, w, dev, mesh):
    """Train the learned start on the GPU (outside the timed region) on windows
    of other seeded RBF animations of the same torus, and register it."""
    import numpy as np
    import torch
    from paper_2111_10105_amd import learned as L
    from synth import animate, learned
    t0 = time.perf_counter()
    blocks = []
    for seed in range(5000, 5006):
        fr = torch.from_numpy(animate.rbf_skinning(w.verts, w.F, 6 + seed % 7, seed=seed,
                                                   dtype=np.float32)).to(dev)
        for w0 in range(0, w.F, w.T):
            blocks.append(dmc.autocorrelation(ctx, mesh, fr[w0:w0 + w.T].contiguous(),
                                              dmc.FP32).cpu().numpy())
    R = np.concatenate(blocks)
    R = R[np.random.default_rng(0).permutation(R.shape[0])]
    omega = learned.sketch_omega(w.T, FIRST_START_SEED + 100)
    k = min(w.k, w.T)
    data = L.Dataset(ctx, R, omega, k)
    theta, hist = L.train(ctx, data, learned.mlp_init(k, FIRST_START_SEED + 200), steps=400,
                          batch=24, lr=2e-3)
    dmc.learned_start(ctx, w.T, k, data.omega, theta)
    ctx._bench_learned = (data, theta)
    return {"blocks": int(R.shape[0]), "steps": 400, "loss_first": round(hist[0][1], 4),
            "loss_last": round(hist[-1][1], 4), "seconds": round(time.perf_counter() - t0, 2),
            "data": "seeded RBF animations 5000-5005 of the same torus"}


def _timed(fn, steps, warmup):
    import torch
    for _ in range(max(1, warmup)):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def bench_icosphere7(args):
    """Icosphere level 7 (163,842 vertices), 512 frames in windows of 64,
    k = 32, 10-bit codes, 1,638 anchors: the float32 form and the precision
    form (bfloat16 covariance and C.Q) with the chained start."""
    import numpy as np
    import torch
    from paper_2111_10105_amd import dmc
    from synth import animate, configs
    t0 = time.perf_counter()
    w = configs.icosphere7()
    gen_s = time.perf_counter() - t0
    n, F, T = w.n, w.F, w.T
    dev = torch.device("cuda:0")
    frames = torch.from_numpy(w.frames).to(dev)
    q0 = torch.from_numpy(animate.gaussian_subspace(T, w.k, FIRST_START_SEED).astype(np.float32)).to(dev)
    ctx = dmc.Context(0)
    t0 = time.perf_counter()
    mesh = dmc.Mesh(ctx, n, w.tris, w.anchors)
    setup_s = time.perf_counter() - t0
    out = {}
    steps = max(1, min(args.steps, 5))
    for name, prec in (("fp32", dmc.FP32), ("bf16", dmc.BF16)):
        p = dmc.make_params(w.k, coef_bits=w.bits, precision=prec)
        codes = torch.empty(dmc.sequence_code_bytes(n, F, T, mesh.nc, p), dtype=torch.uint8,
                            device=dev)
        o = torch.empty_like(frames)
        sec = _timed(lambda: dmc.compress_sequence(ctx, mesh, frames, T, p, q_start=q0, codes=codes,
                                                   out=o, stats=False), steps, 1)
        _, _, st, status = dmc.compress_sequence(ctx, mesh, frames, T, p, q_start=q0, codes=codes,
                                                 out=o, stats=True)
        torch.cuda.synchronize()
        enc = _timed(lambda: dmc.compress_sequence(ctx, mesh, frames, T, p, q_start=q0, codes=codes,
                                                   decode=False, stats=False), steps, 1)
        out[name] = {"ms_per_step": round(sec * 1e3, 3), "value": round(n * F / sec, 1),
                     "encode_ms": round(enc * 1e3, 3),
                     "oi_sweeps_total": int(sum(sum(x["oi_sweeps"]) for x in st)),
                     "cg_resid": st[0]["cg_resid"], "status": status,
                     "nmse_vs_input": nmse(o.cpu().numpy(), w.frames)}
    print(json.dumps({"workload": w.name, "vertices": n, "frames": F, "window": T, "k": w.k,
                      "bits": w.bits, "anchors": int(mesh.nc), "generate_s": round(gen_s, 1),
                      "setup_s": round(setup_s, 2), "factor": mesh.factor_info(), "steps": steps,
                      "forms": out, "unit": "vertex-frames/s", "data": "synthetic"}))
    ctx.close()


def bench_batched(args):
    """64 independent sequences (tori and icospheres of 2k-60k vertices,
    16-128 frames, k in {8, 16, 32}, T = 2k, 1% anchors, float32) encoded and
    decoded by one replayed HIP graph."""
    import torch
    from paper_2111_10105_amd import dmc
    from synth import configs
    t0 = time.perf_counter()
    ws = configs.batched()
    gen_s = time.perf_counter() - t0
    ctx = dmc.Context(0)
    t0 = time.perf_counter()
    meshes = [dmc.Mesh(ctx, w.n, w.tris, w.anchors) for w in ws]
    setup_s = time.perf_counter() - t0
    frames = [torch.from_numpy(w.frames).cuda() for w in ws]
    params = [dmc.make_params(w.k, coef_bits=w.bits, precision=dmc.FP32, init=dmc.INIT_EXACT,
                              cg_max_iters=1) for w in ws]
    t0 = time.perf_counter()
    b = dmc.Batch(ctx, meshes, frames, [w.T for w in ws], params)
    plan_s = time.perf_counter() - t0
    b.run()
    torch.cuda.synchronize()
    sec = _timed(b.run, max(1, min(args.steps, 10)), 1)
    vf = sum(w.n * w.F for w in ws)
    conv = [b.stats(i)[1] == 0 for i in range(len(ws))]
    err = [nmse(b.out[i].cpu().numpy(), ws[i].frames) for i in range(len(ws))]
    print(json.dumps({"workload": "batched-64", "sequences": len(ws), "vertex_frames": vf,
                      "ms_per_run": round(sec * 1e3, 3), "value": round(vf / sec, 1),
                      "unit": "vertex-frames/s", "generate_s": round(gen_s, 1),
                      "setup_s": round(setup_s, 2), "plan_s": round(plan_s, 2),
                      "all_converged": bool(all(conv)), "nmse_vs_input_max": max(err),
                      "tuning": [b.tuning(i) for i in range(len(ws))][:8], "data": "synthetic"}))
    b.close()
    ctx.close()


def nmse(x, y) -> float:
    """sum (x - y)^2 / sum y^2 over every vertex, frame and coordinate."""
    import numpy as np
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    return float(np.sum((x - y) ** 2) / np.sum(y ** 2))


def copy_calibration(mb: float):
    import torch
    nbytes = int(mb * 1e6) // 8 * 8
    x = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
    y = torch.empty_like(x)
    for _ in range(5):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_read": nbytes, "bytes_written": nbytes,
                      "launches": 5}))


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures a single GPU; --gpus {args.gpus} is not supported "
              "(multi-GPU sharding is a design note only)", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration > 0:
        copy_calibration(args.copy_calibration)
        return
    if args.workload == "icosphere7":
        bench_icosphere7(args)
        return
    if args.workload == "batched":
        bench_batched(args)
        return
    import numpy as np
    import torch

    from paper_2111_10105_amd import dmc
    from synth import animate, configs

    w = configs.torus_fp32()
    n, F, T = w.n, w.F, w.T
    dev = torch.device("cuda:0")
    frames = torch.from_numpy(w.frames).to(dev)
    q0_host = animate.gaussian_subspace(T, w.k, FIRST_START_SEED).astype(np.float32)
    q0 = torch.from_numpy(q0_host).to(dev)
    ctx = dmc.Context(0)
    t0 = time.perf_counter()
    mesh = dmc.Mesh(ctx, n, w.tris, w.anchors)
    setup_s = time.perf_counter() - t0
    finfo = mesh.factor_info()
    p = dmc.make_params(w.k, coef_bits=w.bits, precision=dmc.FP32)
    codes = torch.empty(dmc.sequence_code_bytes(n, F, T, mesh.nc, p), dtype=torch.uint8, device=dev)
    out = torch.empty_like(frames)

    def step(stats=False):
        return dmc.compress_sequence(ctx, mesh, frames, T, p, q_start=q0, codes=codes, out=out,
                                     stats=stats)

    for _ in range(max(args.warmup, 1)):
        step()
    torch.cuda.synchronize()
    _, _, stats, status = step(stats=True)
    sweeps_total = sum(sum(s["oi_sweeps"]) for s in stats)
    nw = len(stats)

    # per-family breakdown (HIP events around every launch; outside the timed region)
    fam_steps = 2
    breakdown = {}
    for fam in dmc.KERNELS:
        dmc.profile_start(fam)
        for _ in range(fam_steps):
            step()
        launches, ms = dmc.profile_stop()
        if launches:
            breakdown[fam] = {"ms_per_step": ms / fam_steps, "launches_per_step": launches // fam_steps}
    dominant = max(breakdown, key=lambda f: breakdown[f]["ms_per_step"])
    prof_family = args.profile_kernel or dominant

    # timed region; the profiled family is timed live on the library's stream
    dmc.profile_start(prof_family)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    launches, kernel_ms = dmc.profile_stop()

    # encode-only and decode-only split (outside the timed region)
    def split_time(fn, reps=10):
        fn()  # warm
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / reps * 1e3

    enc_ms = split_time(lambda: dmc.compress_sequence(ctx, mesh, frames, T, p, q_start=q0,
                                                      codes=codes, decode=False, stats=False))
    dec_ms = split_time(lambda: dmc.decode_sequence(ctx, mesh, codes, F, T, p, out=out))

    step()
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    vf = n * F
    value = vf * args.steps / elapsed

    # the other starts of the orthogonal iterations (outside the timed region):
    # per-window Gaussian blocks and the sketch R_c Omega run every window
    # concurrently; exact = per-window eigen-decomposition (Eq. 5)
    nwf = F // T
    variants = {
        "random": (dmc.INIT_RANDOM, torch.from_numpy(np.stack(
            [animate.gaussian_subspace(T, w.k, FIRST_START_SEED + 1 + i) for i in range(nwf)]
        ).astype(np.float32)).to(dev)),
        "sketch": (dmc.INIT_SKETCH, torch.from_numpy(
            animate.gaussian_subspace(T, w.k, FIRST_START_SEED)[0].astype(np.float32)).to(dev)),
        "exact": (dmc.INIT_EXACT, None),
        "learned": (dmc.INIT_LEARNED, None),
    }
    train_info = train_learned_start(ctx, dmc, w, dev, mesh)
    by_init = {}
    for name, (mode, qs) in variants.items():
        pv = dmc.make_params(w.k, coef_bits=w.bits, precision=dmc.FP32, init=mode)
        outv = torch.empty_like(frames)
        for _ in range(2):
            dmc.compress_sequence(ctx, mesh, frames, T, pv, q_start=qs, codes=codes, out=outv,
                                  stats=False)
        torch.cuda.synchronize()
        tv = time.perf_counter()
        nrep = max(3, args.steps // 2)
        for _ in range(nrep):
            dmc.compress_sequence(ctx, mesh, frames, T, pv, q_start=qs, codes=codes, out=outv,
                                  stats=False)
        torch.cuda.synchronize()
        msv = (time.perf_counter() - tv) / nrep * 1e3
        _, _, stv, _ = dmc.compress_sequence(ctx, mesh, frames, T, pv, q_start=qs, codes=codes,
                                             out=outv, stats=True)
        torch.cuda.synchronize()
        by_init[name] = {"ms_per_step": round(msv, 4), "value": round(vf / (msv * 1e-3), 1),
                         "oi_sweeps_total": int(sum(sum(x["oi_sweeps"]) for x in stv)),
                         "nmse_vs_input": nmse(outv.cpu().numpy(), w.frames)}
    by_init["learned"]["training"] = train_info
    dmc.learned_start(ctx, 0, 0, None, None)

    # the precision form (bfloat16 covariance and C.Q, float32 accumulation)
    # with the same chained start, outside the timed region
    pb = dmc.make_params(w.k, coef_bits=w.bits, precision=dmc.BF16)
    outb = torch.empty_like(frames)
    for _ in range(2):
        dmc.compress_sequence(ctx, mesh, frames, T, pb, q_start=q0, codes=codes, out=outb,
                              stats=False)
    torch.cuda.synchronize()
    tb = time.perf_counter()
    nrep = max(3, args.steps // 2)
    for _ in range(nrep):
        dmc.compress_sequence(ctx, mesh, frames, T, pb, q_start=q0, codes=codes, out=outb,
                              stats=False)
    torch.cuda.synchronize()
    msb = (time.perf_counter() - tb) / nrep * 1e3
    _, _, stb, _ = dmc.compress_sequence(ctx, mesh, frames, T, pb, q_start=q0, codes=codes,
                                         out=outb, stats=True)
    torch.cuda.synchronize()
    got_bf16 = outb.cpu().numpy()
    by_precision = {"bf16": {"ms_per_step": round(msb, 4), "value": round(vf / (msb * 1e-3), 1),
                             "oi_sweeps_total": int(sum(sum(x["oi_sweeps"]) for x in stb)),
                             "nmse_vs_input": nmse(got_bf16, w.frames)}}

    # the decode form the library takes (its cost rule, include/dmc.h)
    nz = 3 * min(w.k, T) * nw
    S, A = 16.0 * finfo["solve_entries"], 2.0 * n * mesh.nc
    reduced = mesh.anchor_response()[0] and nz * S + 3 * F * A < 3 * F * S
    model = dict(n=n, F=F, T=T, k=min(w.k, T), nw=nw, rs=4,
                 ncols=nz if reduced else 3 * F, nnz=mesh.nnz,
                 m_nnz=mesh.normal_nnz, finfo=finfo, sweeps_total=sweeps_total, reduced=reduced,
                 nc=int(mesh.nc))
    kernels = {}
    for fam, b in breakdown.items():
        bound, amount, unit = work_model(fam, **model)
        e = {"ms_per_step": round(b["ms_per_step"], 4), "launches_per_step": b["launches_per_step"]}
        if bound:
            if unit == "B":
                ach = amount / (b["ms_per_step"] * 1e-3) / 1e9
                e.update(bound="hbm", achieved_GBs=round(ach, 1), frac=round(ach / HBM_PEAK_GBS, 4))
            else:
                ach = amount / (b["ms_per_step"] * 1e-3) / 1e12
                e.update(bound="mfma", achieved_TFLOPs=round(ach, 3),
                         frac=round(ach / FP64_PEAK_TFLOPS, 5))
        kernels[fam] = e

    roof = None
    if launches:
        bound, amount, unit = work_model(prof_family, **model)
        per_launch = amount / breakdown[prof_family]["launches_per_step"] if amount else None
        avg_s = kernel_ms / launches * 1e-3
        traffic = measured_traffic(prof_family)
        if bound == "hbm":
            ach = per_launch / avg_s / 1e9
            roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(ach / HBM_PEAK_GBS, 4)}
        elif bound == "mfma":
            ach = per_launch / avg_s / 1e12
            roof = {"bound": "mfma", "achieved": round(ach, 3), "peak": FP64_PEAK_TFLOPS,
                    "unit": "TFLOP/s", "frac": round(ach / FP64_PEAK_TFLOPS, 5)}
        if roof is not None:
            roof.update(traffic=traffic, kernel=prof_family, launches=launches,
                        avg_us=round(kernel_ms / launches * 1e3, 2),
                        algorithmic_per_launch=per_launch, dtype="f64")

    result = {
        "metric": "vertex-frames/s encode+decode at fixed NMSE",
        "value": round(value, 1),
        "unit": "vertex-frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32/f64",
        "data": "synthetic",
        "config": {"workload": w.name, "vertices": n, "frames": F, "window": T, "k": w.k,
                   "bits": w.bits, "anchors": int(mesh.nc), "first_start": "gaussian",
                   "oi_tol": p.oi_tol, "precond": "cholesky", "cg_tol": p.cg_tol},
        "split_ms": {"encode": round(enc_ms, 3), "decode": round(dec_ms, 3)},
        "cg_iters": stats[0]["cg_iters"],
        "oi_sweeps": [s["oi_sweeps"] for s in stats],
        "setup_s": round(setup_s, 3),
        "factor": {kk: (round(v, 4) if isinstance(v, float) else v) for kk, v in finfo.items()},
        "status": status,
        "roofline": roof,
        "kernels": kernels,
        "by_init": by_init,
        "by_precision": by_precision,
    }

    result["nmse_vs_input"] = nmse(got, w.frames)
    if not args.no_cpu_baseline:
        import oracle as O
        # the float64 oracle on the host cores, over the same whole sequence
        # (same first start block, as float64 of the float32 values)
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        tc = time.perf_counter()
        _, ref = O.compress_sequence(n, w.tris, w.frames, w.anchors, T, w.k, w.bits,
                                     first_start=q0_host.astype(np.float64), fp32_data=True)
        cpu_s = time.perf_counter() - tc
        result["cpu_baseline"] = {"value": round(vf / cpu_s, 1), "unit": "vertex-frames/s",
                                  "cores": threads, "kind": "oracle",
                                  "sample": f"whole workload once ({n} vertices x {F} frames, "
                                            f"{cpu_s:.1f} s)"}
        result["nmse_vs_oracle"] = nmse(got, ref)
        result["oracle_nmse_vs_input"] = nmse(ref, w.frames)
        result["fixed_nmse_ok"] = bool(result["nmse_vs_oracle"] <= 1e-5 and
                                       result["nmse_vs_input"] <= 1.01 * result["oracle_nmse_vs_input"])
        for v in by_init.values():
            v["within_1pct_of_oracle_nmse"] = bool(
                v["nmse_vs_input"] <= 1.01 * result["oracle_nmse_vs_input"])
        bf = by_precision["bf16"]
        bf["nmse_vs_oracle"] = nmse(got_bf16, ref)
        bf["within_1pct_of_oracle_nmse"] = bool(
            bf["nmse_vs_input"] <= 1.01 * result["oracle_nmse_vs_input"])
    print(json.dumps(result))
    ctx.close()


if __name__ == "__main__":
    main()
