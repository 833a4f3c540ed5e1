"""Benchmark: vertex-frames per second of encode + decode on one MI355X.

One step = the whole path over one synthetic sequence already resident in
HBM: delta coordinates, autocorrelation, orthogonal iterations with the Ritz
step, projection + quantisation, anchors (encode), then back-projection and the
anchored least-squares solve by preconditioned conjugate gradients on the
normal equations, and the frames (decode).

Workload (the largest single-GPU configuration): icosphere level 7 (163,842
vertices), 512 frames in windows of 64, 8-bone Gaussian-RBF skinning, k = 32,
10-bit codes, 1,638 anchors (1%), float32 frames.  The first window's
orthogonal iterations start from a seeded Gaussian block, every later window
from the previous window's subspace (Algorithm 1).  The precision form
(bfloat16 covariance and C.Q) and the other starts run beside it, and the
128 x 128 torus (16,384 vertices, 256 frames, T = 32, k = 16, 12 bits, 64
anchors) as a second workload.

Each timed step is bracketed by device synchronisations and preceded,
outside its bracket, by a 512 MB device write that evicts the frames from
the 256 MB last-level cache (MALL).  The one-off mesh set-up (CSR pattern,
normal matrix and its Cholesky factor on the host) is reported as setup_s and
in a set-up-inclusive rate for one sequence.

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
FP32_PEAK_TFLOPS = 157.3   # MI355X FP32 matrix, TFLOP/s
FIRST_START_SEED = 909     # seeded Gaussian start block of window 0
MALL_FLUSH_BYTES = 512 << 20

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
                 "delta": "k_delta", "back_project": "k_coef_rows", "rhs": "k_rhs_expand"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-kernel", default=None,
                    help="kernel family timed live (default: the dominant one)")
    ap.add_argument("--copy-calibration", type=float, default=0.0, metavar="MB")
    ap.add_argument("--workload", default="icosphere7",
                    choices=["torus", "icosphere7", "batched", "rd", "learned"],
                    help="icosphere7: the headline workload (level 7, 512 frames); torus: the "
                         "128 x 128 torus alone; batched: 64 sequences in one graph; rd: the "
                         "rate-distortion sweep over k; learned: the learned start trained on "
                         "2,000 windows of 8-16-bone animations of 10k-160k-vertex meshes and "
                         "compared with the plain starts on held-out seeds")
    ap.add_argument("--no-second-workload", action="store_true",
                    help="skip the torus workload that runs beside the headline")
    ap.add_argument("--headline-only", action="store_true",
                    help="time the headline steps and kernel families only (no start or "
                         "precision variants, no second workload, no CPU baseline): the run "
                         "profiled under rocprofv3")
    return ap.parse_args()


def source_hash(family: str) -> str:
    path = os.path.join(ROOT, "paper_2111_10105_amd", "csrc", FAMILY_SOURCE[family])
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(family: str, workload: str):
    """HBM bytes per launch of `family` from the committed counter summary
    (profiles/<kernel>_<workload prefix>_pmc.txt), or None when there is none
    or the kernel source changed since the counters were taken."""
    kern = FAMILY_KERNEL.get(family)
    if kern is None:
        return None
    tag = "icosphere7" if workload.startswith("icosphere7") else "torus128"
    path = os.path.join(ROOT, "profiles", f"{kern}_{tag}_pmc.txt")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_hash = re.search(r"^source_sha256_16:\s*(\S+)", text, re.M)
    m_bytes = re.search(r"^hbm_bytes_per_launch:\s*(\S+)", text, re.M)
    if not m_hash or not m_bytes or m_hash.group(1) != source_hash(family):
        return None
    return float(m_bytes.group(1))


def work_model(fam, *, n, F, T, k, nw, rs, ncols, nnz, m_nnz, finfo, sweeps_total, reduced=False,
               nc=0, cg_first=True):
    """Algorithmic work of one step for a kernel family: (bound, amount, unit,
    peak) with amount in bytes (hbm) or flops (mfma) and the peak of that
    roof.  Bytes count each input read once and each output written once;
    flops count 2 per multiply-add of the operation's definition.  ncols:
    columns of the decoder's solve (3k per window with the mesh's anchor
    response, `reduced`, else 3F); nc anchors; cg_first: every update of the
    step is the first of its solve (x taken as zero: 5 vectors, else 6)."""
    vec = 8.0 * n * ncols                     # one float64 n x ncols block
    fr = float(rs) * 3 * n * F                # the frames (or deltas) in their type
    coef = 3.0 * k * n * nw
    hbm, f64 = HBM_PEAK_GBS, FP64_PEAK_TFLOPS
    if fam == "delta":
        return "hbm", 2 * fr + 4.0 * (nnz + n + 1), "B", hbm
    if fam == "autocorr":
        return "hbm", fr, "B", hbm
    if fam == "oi":
        per = 2.0 * T * T * k + 2.0 * T * k * k + k ** 3 / 3.0
        return "mfma", per * sweeps_total, "flop", f64
    if fam == "project":
        return "hbm", fr + rs * coef, "B", hbm
    if fam == "quantise":
        return "hbm", rs * coef + 2.0 * coef, "B", hbm
    if fam == "anchors":
        return "hbm", 2.0 * rs * 3 * nc * F, "B", hbm
    if fam == "back_project":  # the dequantised coefficient rows (float64)
        return "hbm", 2.0 * coef + 8.0 * coef, "B", hbm
    if fam == "rhs":  # L^T on the coefficient rows (and, direct form, their expansion)
        return "hbm", 8.0 * coef + vec, "B", hbm
    if fam == "cg_spmm":
        return "hbm", 2 * vec + 12.0 * m_nnz, "B", hbm
    if fam == "cg_update":
        return "hbm", (5 if cg_first else 6) * vec, "B", hbm
    if fam == "chol_fwd_gather":
        # rows above the leaves: read r, write W; plus the update rows read
        gathered = float(n) - finfo["leaf_rows"]
        return "hbm", 8.0 * (2 * gathered + finfo["update_rows"]) * ncols, "B", hbm
    if fam in ("chol_fwd_solve", "chol_bwd_solve"):
        return "mfma", 2.0 * finfo["solve_entries"] * ncols, "flop", f64
    if fam == "to_frames":
        if reduced:  # X = Z U~^T + G A^ per window and coordinate, written as frames
            return ("mfma", 2.0 * n * 3 * F * (nc + k), "flop",
                    FP32_PEAK_TFLOPS if rs == 4 else f64)
        return "hbm", vec + fr, "B", hbm
    return None, None, None, None


def host_description():
    """CPU model, logical CPUs and the BLAS libraries numpy uses (with their
    default thread counts, outside any limit) of the machine the benchmark
    runs on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    blas = []
    try:
        from threadpoolctl import threadpool_info
        blas = [{"api": i.get("internal_api"), "threads": i.get("num_threads")}
                for i in threadpool_info()]
    except Exception:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(), "blas_default_threads": blas}


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


def bench_batched(args):
    """64 independent sequences (tori and icospheres of 2k-60k vertices,
    16-128 frames, k in {8, 16, 32}, T = 2k, 1% anchors, float32) encoded and
    decoded by one replayed HIP graph."""
    import torch
    import numpy as np
    from paper_2111_10105_amd import dmc
    from synth import animate, configs
    t0 = time.perf_counter()
    ws = configs.batched()
    gen_s = time.perf_counter() - t0
    ctx = dmc.Context(0)
    t0 = time.perf_counter()
    meshes = [dmc.Mesh(ctx, w.n, w.tris, w.anchors) for w in ws]
    setup_s = time.perf_counter() - t0
    frames = [torch.from_numpy(w.frames).cuda() for w in ws]
    # every window starts from its sketch R_c Omega (one Gaussian Omega per
    # sequence), so all windows of all sequences are independent
    params = [dmc.make_params(w.k, coef_bits=w.bits, precision=dmc.FP32, init=dmc.INIT_SKETCH,
                              cg_max_iters=1) for w in ws]
    omegas = [torch.from_numpy(animate.gaussian_subspace(w.T, w.k, 4500 + i)[0]
                               .astype(np.float32)).cuda() for i, w in enumerate(ws)]
    t0 = time.perf_counter()
    b = dmc.Batch(ctx, meshes, frames, [w.T for w in ws], params, q_starts=omegas)
    plan_s = time.perf_counter() - t0
    b.run()
    torch.cuda.synchronize()
    sec = _timed(b.run, max(1, min(args.steps, 10)), 1)
    vf = sum(w.n * w.F for w in ws)
    conv = [b.stats(i)[1] == 0 for i in range(len(ws))]
    err = [nmse(b.out[i].cpu().numpy(), ws[i].frames) for i in range(len(ws))]
    print(json.dumps({"workload": "batched-64", "sequences": len(ws), "vertex_frames": vf,
                      "start": "sketch",
                      "ms_per_run": round(sec * 1e3, 3), "value": round(vf / sec, 1),
                      "value_incl_setup": round(vf / (sec + setup_s + plan_s), 1),
                      "unit": "vertex-frames/s", "generate_s": round(gen_s, 1),
                      "setup_s": round(setup_s, 2), "plan_s": round(plan_s, 2),
                      "all_converged": bool(all(conv)), "nmse_vs_input_max": max(err),
                      "tuning": [b.tuning(i) for i in range(len(ws))][:8], "data": "synthetic"}))
    b.close()
    ctx.close()


def bench_learned(args):
    """The learned start at its training configuration: 2,000 windows of 64
    frames of seeded 8-16-bone RBF animations of six meshes of 10k-160k
    vertices (250 animations of 512 frames, skinned on the GPU), covariances
    by the library, targets the exact eigenvectors (k = 32); trained on the
    GPU; then on held-out seeds, sweeps of Algorithm 1 to its tolerance from
    the learned start, a seeded Gaussian block and the previous window's
    subspace, over all blocks and over those whose numerical rank exceeds k."""
    import numpy as np
    import torch
    from paper_2111_10105_amd import dmc
    from paper_2111_10105_amd import learned as L
    from synth import animate, learned, meshes
    T, k, nwin = 64, 32, 8
    t_all = time.perf_counter()
    ctx = dmc.Context(0)
    dev = torch.device("cuda:0")
    shapes = [("icosphere5", meshes.icosphere(5)), ("torus160x128", meshes.torus(160, 128)),
              ("icosphere6", meshes.icosphere(6)), ("torus256x256", meshes.torus(256, 256)),
              ("torus400x250", meshes.torus(400, 250)), ("icosphere7", meshes.icosphere(7))]
    mlist = []
    for name, (v, t) in shapes:
        n = v.shape[0]
        mlist.append((name, v, dmc.Mesh(ctx, n, t, animate.choose_anchors(n, 8, seed=1))))

    def windows(seeds):
        """[nb][T][T] covariances (coordinate blocks of each window in order),
        numerical ranks, and (animation, window, coordinate) of each block."""
        R, meta = [], []
        for a, seed in enumerate(seeds):
            name, v, mesh = mlist[a % len(mlist)]
            bones = 8 + seed % 9
            fr = animate.rbf_skinning_torch(v, T * nwin, bones, seed, dev)
            for w in range(nwin):
                Rw = dmc.autocorrelation(ctx, mesh, fr[w * T:(w + 1) * T].contiguous(), dmc.FP32)
                R.append(Rw.cpu().numpy())
                meta += [(a, w, c, bones, name) for c in range(3)]
            del fr
        R = np.concatenate(R)
        ev = np.linalg.eigvalsh(R)
        rank = (ev > 1e-13 * ev[:, -1:]).sum(axis=1)
        return R, rank, meta

    t0 = time.perf_counter()
    R_train, rank_train, _ = windows(list(range(20000, 20250)))
    gen_s = time.perf_counter() - t0
    omega = learned.sketch_omega(T, 7001)
    R_test, rank_test, meta = windows(list(range(90000, 90024)))
    nb = R_test.shape[0]

    def summ(x, mask=None):
        x = np.asarray(x, dtype=np.float64)
        if mask is not None:
            x = x[mask]
        if x.size == 0:
            return None
        return {"mean": round(float(x.mean()), 3), "median": float(np.median(x)),
                "max": float(x.max()), "blocks": int(x.size)}

    def train_and_compare(k):
        t0 = time.perf_counter()
        perm = np.random.default_rng(0).permutation(R_train.shape[0])
        data = L.Dataset(ctx, R_train[perm], omega, k)
        steps = max(200, 15 * args.steps * 10)
        theta, hist = L.train(ctx, data, learned.mlp_init(k, 7002), steps=steps, batch=64,
                              lr=2e-3)
        train_s = time.perf_counter() - t0
        gauss = animate.gaussian_subspace(T, k, 7003)
        starts = np.stack([gauss[i % 3] for i in range(nb)])
        ev = L.evaluate(ctx, R_test, theta, omega, k, random_starts=starts, oi_tol=1e-12,
                        max_sweeps=200)
        # previous window's subspace (same animation and coordinate); window 0
        # of an animation has none and is left out of that column
        exact = dmc.make_params(k, precision=dmc.FP64, init=dmc.INIT_EXACT)
        U, _, _ = dmc.oi_blocks(ctx, torch.from_numpy(R_test).to(dev), exact)
        Uh = U.cpu().numpy()
        prev_idx = [i for i in range(nb) if meta[i][1] > 0]
        prev_start = np.stack([Uh[i - 3] for i in prev_idx])
        pr = dmc.make_params(k, precision=dmc.FP64, init=dmc.INIT_RANDOM, oi_tol=1e-12,
                             oi_max_sweeps=200)
        _, sw_prev, res_prev = dmc.oi_blocks(ctx, torch.from_numpy(R_test[prev_idx]).to(dev), pr,
                                             q_start=torch.from_numpy(prev_start).to(dev))
        above = rank_test > k
        prev_mask = np.zeros(nb, dtype=bool)
        prev_mask[prev_idx] = True
        sw_prev_full = np.full(nb, np.nan)
        sw_prev_full[prev_idx] = sw_prev
        return {
            "k": k,
            "train": {"windows": int(R_train.shape[0] // 3), "blocks": int(R_train.shape[0]),
                      "steps": steps, "batch": 64, "loss_first": round(hist[0][1], 4),
                      "loss_last": round(hist[-1][1], 4), "seconds": round(train_s, 1),
                      "blocks_rank_above_k": int((rank_train > k).sum())},
            "test_blocks_rank_above_k": int(above.sum()),
            "sweeps_all": {"learned": summ(ev["sweeps_learned"]),
                           "gaussian": summ(ev["sweeps_random"]),
                           "previous_window": summ(sw_prev_full, prev_mask)},
            "sweeps_rank_above_k": {"learned": summ(ev["sweeps_learned"], above),
                                    "gaussian": summ(ev["sweeps_random"], above),
                                    "previous_window": summ(sw_prev_full, above & prev_mask)},
            "not_converged": {"learned": int((ev["resid_learned"] > 1e-12).sum()),
                              "gaussian": int((ev["resid_random"] > 1e-12).sum()),
                              "previous_window": int((res_prev > 1e-12).sum())},
            "start_resid_median": {"learned": float(np.median(ev["start_resid_learned"])),
                                   "gaussian": float(np.median(ev["start_resid_random"]))},
        }

    result = {
        "workload": "learned-start-T64", "data": "synthetic (seeded RBF animations, 8-16 bones)",
        "meshes": [(name, int(v.shape[0])) for name, v, _ in mlist],
        "generate_seconds": round(gen_s, 1),
        "test": {"windows": nb // 3, "blocks": nb, "seeds": "90000-90023 (held out)"},
        "oi_tol": 1e-12,
        "by_k": [train_and_compare(32), train_and_compare(16)],
        "seconds": round(time.perf_counter() - t_all, 1),
    }
    print(json.dumps(result))
    ctx.close()


def bench_rd_sweep(args):
    """Rate-distortion sweep in the manner of the paper's Fig. 3 (only the
    first k of the eigen-trajectory rows kept, k in {2, 5, 10, 20, 30}) on a
    synthetic stand-in of its Handstand workload's shape: a 100 x 100 torus
    (10,000 vertices), 175 frames in 5 windows of 35 (the "blocks"
    variant), 6-bone RBF skinning, 12-bit codes, 1% anchors, float32.  Per k:
    bits per vertex per frame and coordinate of the stream (Eq. 13), the
    reconstruction's NMSE against the input and the relative error of its
    delta coordinates (the Laplacian-domain part of a visual error; the
    paper's NMSVE is not defined in its text), and the step time."""
    import numpy as np
    import torch
    from paper_2111_10105_amd import dmc
    from synth import animate, configs, meshes
    v, t = meshes.torus(100, 100)
    F, T = 175, 35
    fr = animate.rbf_skinning(v, F, 6, seed=808, dtype=np.float32)
    anchors = animate.choose_anchors(v.shape[0], 100, seed=809)
    n = v.shape[0]
    ctx = dmc.Context(0)
    mesh = dmc.Mesh(ctx, n, t, anchors)
    frames = torch.from_numpy(fr).cuda()
    delta_in = dmc.delta(ctx, mesh, frames, dmc.FP32).cpu().numpy()
    flush = Flusher()
    rows = []
    for k in (2, 5, 10, 20, 30):
        p = dmc.make_params(k, coef_bits=12, precision=dmc.FP32, init=dmc.INIT_EXACT)
        codes = torch.empty(dmc.sequence_code_bytes(n, F, T, mesh.nc, p), dtype=torch.uint8,
                            device="cuda:0")
        times, st, status, out = run_form(dmc, ctx, mesh, frames, T, p, None, 5, flush, codes)
        got = out.cpu().numpy()
        d_out = dmc.delta(ctx, mesh, out, dmc.FP32).cpu().numpy()
        rows.append({"k": k, "status": status,
                     "bpvf": {key: round(sum(x[key] * x["T"] for x in st) / F, 5)
                              for key in ("q", "q_a", "q_d", "q_s")},
                     "nmse_vs_input": nmse(got, fr),
                     "delta_rel_error": float(np.sqrt(np.sum((d_out - delta_in) ** 2) /
                                                      np.sum(delta_in.astype(np.float64) ** 2))),
                     "ms_per_step": round(sum(times) / len(times) * 1e3, 3)})
    print(json.dumps({"workload": f"torus100x100-{n}v-{F}f-T{T}-b12-rd-sweep",
                      "data": "synthetic (seeded RBF skinning in the shape of Handstand)",
                      "sweep": rows}))
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


class Flusher:
    """A 512 MB device buffer written between timed steps: the frames (and
    everything else) then come from HBM, not from the 256 MB MALL."""

    def __init__(self):
        import torch
        self.buf = torch.empty(MALL_FLUSH_BYTES // 4, dtype=torch.float32, device="cuda:0")
        self.v = 0.0

    def __call__(self):
        self.v += 1.0
        self.buf.fill_(self.v)


def timed_steps(step, steps, flush):
    """Run `steps` steps, each bracketed by device synchronisations and
    preceded (outside its bracket) by a cache flush; returns the list of step
    times in seconds."""
    import torch
    times = []
    for _ in range(steps):
        flush()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        step()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    return times


def family_breakdown(dmc, step, reps=2):
    """Per kernel family: milliseconds and launches per step (HIP events
    around every launch of the family, outside the timed region)."""
    out = {}
    for fam in dmc.KERNELS:
        dmc.profile_start(fam)
        for _ in range(reps):
            step()
        launches, ms = dmc.profile_stop()
        if launches:
            out[fam] = {"ms_per_step": ms / reps, "launches_per_step": launches // reps}
    return out


def kernel_table(breakdown, model):
    kernels = {}
    for fam, b in breakdown.items():
        bound, amount, unit, peak = work_model(fam, **model)
        e = {"ms_per_step": round(b["ms_per_step"], 4), "launches_per_step": b["launches_per_step"]}
        if bound:
            if unit == "B":
                ach = amount / (b["ms_per_step"] * 1e-3) / 1e9
                e.update(bound="hbm", achieved_GBs=round(ach, 1), frac=round(ach / peak, 4))
            else:
                ach = amount / (b["ms_per_step"] * 1e-3) / 1e12
                e.update(bound="mfma", achieved_TFLOPs=round(ach, 3), peak_TFLOPs=peak,
                         frac=round(ach / peak, 5))
        kernels[fam] = e
    return kernels


def run_form(dmc, ctx, mesh, frames, T, p, q0, steps, flush, codes):
    """A form (precision or start) of the path: step time over `steps`
    flushed steps, sweeps and the reconstruction."""
    import torch
    out = torch.empty_like(frames)

    def step():
        dmc.compress_sequence(ctx, mesh, frames, T, p, q_start=q0, codes=codes, out=out,
                              stats=False)
    step()
    times = timed_steps(step, steps, flush)
    _, _, st, status = dmc.compress_sequence(ctx, mesh, frames, T, p, q_start=q0, codes=codes,
                                             out=out, stats=True)
    torch.cuda.synchronize()
    return times, st, status, out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures a single GPU; --gpus {args.gpus} is not supported "
              "(multi-GPU sharding is a design note only)", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration > 0:
        copy_calibration(args.copy_calibration)
        return
    if args.workload == "batched":
        bench_batched(args)
        return
    if args.workload == "rd":
        bench_rd_sweep(args)
        return
    if args.workload == "learned":
        bench_learned(args)
        return
    import numpy as np
    import torch

    from paper_2111_10105_amd import dmc
    from synth import animate, configs

    w = configs.icosphere7() if args.workload == "icosphere7" else configs.torus_fp32()
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
    flush = Flusher()

    def step(stats=False):
        return dmc.compress_sequence(ctx, mesh, frames, T, p, q_start=q0, codes=codes, out=out,
                                     stats=stats)

    for _ in range(max(args.warmup, 1)):
        step()
    torch.cuda.synchronize()
    _, _, stats, status = step(stats=True)
    sweeps_total = sum(sum(s["oi_sweeps"]) for s in stats)
    nw = len(stats)

    breakdown = family_breakdown(dmc, step)
    dominant = max(breakdown, key=lambda f: breakdown[f]["ms_per_step"])
    prof_family = args.profile_kernel or dominant

    # timed region: K steps, each bracketed by synchronisations after a flush;
    # the profiled family is timed live on the library's stream
    dmc.profile_start(prof_family)
    times = timed_steps(step, args.steps, flush)
    launches, kernel_ms = dmc.profile_stop()
    elapsed = sum(times)

    if args.headline_only:
        args.no_second_workload = True
        args.no_cpu_baseline = True
    # encode-only and decode-only split (outside the timed region)
    enc = timed_steps(lambda: dmc.compress_sequence(ctx, mesh, frames, T, p, q_start=q0,
                                                    codes=codes, decode=False, stats=False),
                      5, flush)
    dec = timed_steps(lambda: dmc.decode_sequence(ctx, mesh, codes, F, T, p, out=out), 5, flush)
    step()
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    vf = n * F
    value = vf * args.steps / elapsed
    ms = elapsed / args.steps * 1e3

    # the other starts (per-window Gaussian blocks, the sketch R_c Omega, the
    # exact per-window eigen-decomposition run every window concurrently) and
    # the precision form, outside the timed region
    nwf = F // T
    variants = {
        "random": (dmc.INIT_RANDOM, torch.from_numpy(np.stack(
            [animate.gaussian_subspace(T, w.k, FIRST_START_SEED + 1 + i) for i in range(nwf)]
        ).astype(np.float32)).to(dev)),
        "sketch": (dmc.INIT_SKETCH, torch.from_numpy(
            animate.gaussian_subspace(T, w.k, FIRST_START_SEED)[0].astype(np.float32)).to(dev)),
        "exact": (dmc.INIT_EXACT, None),
    }
    nrep = max(3, args.steps // 4)
    by_init = {}
    if args.headline_only:
        variants = {}
    for name, (mode, qs) in variants.items():
        pv = dmc.make_params(w.k, coef_bits=w.bits, precision=dmc.FP32, init=mode)
        tv, stv, stt, outv = run_form(dmc, ctx, mesh, frames, T, pv, qs, nrep, flush, codes)
        msv = sum(tv) / len(tv) * 1e3
        by_init[name] = {"ms_per_step": round(msv, 4), "value": round(vf / (msv * 1e-3), 1),
                         "oi_sweeps_total": int(sum(sum(x["oi_sweeps"]) for x in stv)),
                         "status": stt, "nmse_vs_input": nmse(outv.cpu().numpy(), w.frames)}
    pb = dmc.make_params(w.k, coef_bits=w.bits, precision=dmc.BF16)
    tb, stb, stt, outb = run_form(dmc, ctx, mesh, frames, T, pb, q0,
                                  1 if args.headline_only else nrep, flush, codes)
    msb = sum(tb) / len(tb) * 1e3
    got_bf16 = outb.cpu().numpy()
    by_precision = {"bf16": {"ms_per_step": round(msb, 4), "value": round(vf / (msb * 1e-3), 1),
                             "oi_sweeps_total": int(sum(sum(x["oi_sweeps"]) for x in stb)),
                             "oi_resid_max": max(max(x["oi_resid"]) for x in stb),
                             "status": stt, "nmse_vs_input": nmse(got_bf16, w.frames)},
                    "fp32": {"oi_sweeps_total": sweeps_total,
                             "oi_resid_max": max(max(x["oi_resid"]) for x in stats)}}

    # the decode form the library takes (its cost rule, include/dmc.h)
    nz = 3 * min(w.k, T) * nw
    S, A = 16.0 * finfo["solve_entries"], 2.0 * n * mesh.nc
    reduced = mesh.anchor_response()[0] and nz * S + 3 * F * A < 3 * F * S
    model = dict(n=n, F=F, T=T, k=min(w.k, T), nw=nw, rs=4,
                 ncols=nz if reduced else 3 * F, nnz=mesh.nnz,
                 m_nnz=mesh.normal_nnz, finfo=finfo, sweeps_total=sweeps_total, reduced=reduced,
                 nc=int(mesh.nc), cg_first=stats[0]["cg_iters"] == 1)
    kernels = kernel_table(breakdown, model)

    roof = None
    if launches:
        bound, amount, unit, peak = work_model(prof_family, **model)
        per_launch = amount / breakdown[prof_family]["launches_per_step"] if amount else None
        avg_s = kernel_ms / launches * 1e-3
        traffic = measured_traffic(prof_family, w.name)
        if bound == "hbm":
            ach = per_launch / avg_s / 1e9
            roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": peak, "unit": "GB/s",
                    "frac": round(ach / peak, 4)}
        elif bound == "mfma":
            ach = per_launch / avg_s / 1e12
            roof = {"bound": "mfma", "achieved": round(ach, 3), "peak": peak,
                    "unit": "TFLOP/s", "frac": round(ach / peak, 5)}
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
        "ms_per_step": round(ms, 4),
        "ms_per_step_median": round(float(np.median(times)) * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32/f64",
        "data": "synthetic",
        "config": {"workload": w.name, "vertices": n, "frames": F, "window": T, "k": w.k,
                   "bits": w.bits, "anchors": int(mesh.nc), "first_start": "gaussian",
                   "oi_tol": p.oi_tol, "precond": "cholesky", "cg_tol": p.cg_tol,
                   "decode_form": "reduced" if reduced else "direct",
                   "mall_flush_bytes": MALL_FLUSH_BYTES},
        "setup_s": round(setup_s, 3),
        "value_incl_setup": round(vf / (ms * 1e-3 + setup_s), 1),
        "split_ms": {"encode": round(sum(enc) / len(enc) * 1e3, 3),
                     "decode": round(sum(dec) / len(dec) * 1e3, 3)},
        "cg_iters": stats[0]["cg_iters"],
        "oi_sweeps": [s["oi_sweeps"] for s in stats],
        "bpvf": {key: round(sum(s[key] * s["T"] for s in stats) / F, 5)
                 for key in ("q", "q_a", "q_d", "q_s")},
        "factor": {kk: (round(v, 4) if isinstance(v, float) else v) for kk, v in finfo.items()},
        "status": status,
        "roofline": roof,
        "kernels": kernels,
        "by_init": by_init,
        "by_precision": by_precision,
    }
    result["nmse_vs_input"] = nmse(got, w.frames)

    if args.workload == "icosphere7" and not args.no_second_workload:
        result["torus128"] = bench_torus(dmc, ctx, flush, args)

    if not args.no_cpu_baseline:
        import oracle as O
        from threadpoolctl import threadpool_limits
        # the float64 oracle on the host, on the first window of the same
        # workload (same first start block, as float64 of the float32
        # values); its sparse LU, Jacobi sweeps and quantiser loops are
        # single-threaded, so it runs with one BLAS thread
        Ts = min(T, F)
        with threadpool_limits(limits=1):
            tc = time.perf_counter()
            _, ref = O.compress_sequence(n, w.tris, w.frames[:Ts], w.anchors, T, w.k, w.bits,
                                         first_start=q0_host.astype(np.float64), fp32_data=True)
            cpu_s = time.perf_counter() - tc
        result["cpu_baseline"] = {"value": round(n * Ts / cpu_s, 1), "unit": "vertex-frames/s",
                                  "cores": 1, "kind": "oracle", "blas_threads_used": 1,
                                  "sample": f"first window of the workload ({n} vertices x {Ts} "
                                            f"frames, encode + decode incl. its sparse LU, "
                                            f"{cpu_s:.1f} s)",
                                  "host": host_description()}
        # fixed NMSE: the GPU's first window (the chain starts from the same
        # block) against the oracle's
        g0, f0 = got[:Ts], w.frames[:Ts]
        result["nmse_vs_oracle_window0"] = nmse(g0, ref)
        result["oracle_nmse_vs_input_window0"] = nmse(ref, f0)
        result["gpu_nmse_vs_input_window0"] = nmse(g0, f0)
        result["fixed_nmse_ok"] = bool(result["nmse_vs_oracle_window0"] <= 1e-5 and
                                       result["gpu_nmse_vs_input_window0"] <=
                                       1.01 * result["oracle_nmse_vs_input_window0"])
        bf = by_precision["bf16"]
        bf["nmse_vs_oracle_window0"] = nmse(got_bf16[:Ts], ref)
        bf["nmse_vs_input_window0"] = nmse(got_bf16[:Ts], f0)
        bf["within_1pct_of_oracle_nmse"] = bool(
            bf["nmse_vs_input_window0"] <= 1.01 * result["oracle_nmse_vs_input_window0"])
    print(json.dumps(result))
    ctx.close()


def bench_torus(dmc, ctx, flush, args):
    """The 128 x 128 torus workload (16,384 vertices, 256 frames in windows of
    32, k = 16, 12 bits, 64 anchors, float32, chained start) with its NMSE
    against the float64 oracle over the whole sequence."""
    import numpy as np
    import torch
    from synth import animate, configs
    w = configs.torus_fp32()
    n, F, T = w.n, w.F, w.T
    dev = torch.device("cuda:0")
    frames = torch.from_numpy(w.frames).to(dev)
    q0_host = animate.gaussian_subspace(T, w.k, FIRST_START_SEED).astype(np.float32)
    q0 = torch.from_numpy(q0_host).to(dev)
    t0 = time.perf_counter()
    mesh = dmc.Mesh(ctx, n, w.tris, w.anchors)
    setup_s = time.perf_counter() - t0
    p = dmc.make_params(w.k, coef_bits=w.bits, precision=dmc.FP32)
    codes = torch.empty(dmc.sequence_code_bytes(n, F, T, mesh.nc, p), dtype=torch.uint8, device=dev)
    times, st, status, out = run_form(dmc, ctx, mesh, frames, T, p, q0, max(5, args.steps), flush,
                                      codes)
    ms = sum(times) / len(times) * 1e3
    res = {"workload": w.name, "ms_per_step": round(ms, 4), "value": round(n * F / (ms * 1e-3), 1),
           "setup_s": round(setup_s, 3),
           "value_incl_setup": round(n * F / (ms * 1e-3 + setup_s), 1), "status": status,
           "oi_sweeps_total": int(sum(sum(x["oi_sweeps"]) for x in st)),
           "nmse_vs_input": nmse(out.cpu().numpy(), w.frames)}
    if not args.no_cpu_baseline:
        import oracle as O
        _, ref = O.compress_sequence(n, w.tris, w.frames, w.anchors, T, w.k, w.bits,
                                     first_start=q0_host.astype(np.float64), fp32_data=True)
        got = out.cpu().numpy()
        res["nmse_vs_oracle"] = nmse(got, ref)
        res["oracle_nmse_vs_input"] = nmse(ref, w.frames)
        res["fixed_nmse_ok"] = bool(res["nmse_vs_oracle"] <= 1e-5 and
                                    res["nmse_vs_input"] <= 1.01 * res["oracle_nmse_vs_input"])
    return res


if __name__ == "__main__":
    main()
