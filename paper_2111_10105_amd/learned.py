"""Training and use of the learned start of the orthogonal iterations.

The network (a row-wise perceptron on the sketch R Omega of a window's
autocorrelation, see include/dmc.h) is trained on the GPU by the library's own
forward, loss, backward and Adam kernels, on the subspaces U_k the plain method
converges to (exact eigenvectors of each block).  This module only orders the
calls and the data: every arithmetic step runs in the HIP library.
"""
from __future__ import annotations

import numpy as np

from . import dmc


class Dataset:
    """Training blocks on the device: sketches S [nb][T][32] (float32) and
    targets U [nb][T][k] (float64), in the order given."""

    def __init__(self, ctx: dmc.Context, R_host: np.ndarray, omega_host: np.ndarray, k: int):
        import torch
        R_host = np.ascontiguousarray(R_host, dtype=np.float64)
        nb, T, _ = R_host.shape
        self.nb, self.T, self.k = nb, T, k
        self.R = torch.from_numpy(R_host).cuda()
        self.omega = torch.from_numpy(np.ascontiguousarray(omega_host, dtype=np.float64)).cuda()
        self.S = dmc.mlp_sketch(ctx, self.R, self.omega)
        p = dmc.make_params(k, precision=dmc.FP64, init=dmc.INIT_EXACT)
        self.U, _, _ = dmc.oi_blocks(ctx, self.R, p)


def train(ctx: dmc.Context, data: Dataset, theta0: np.ndarray, *, steps: int, batch: int,
          lr: float = 1e-3, mu: float = 0.1, log_every: int = 50):
    """Adam on minibatches of `batch` consecutive blocks (cycling through the
    data set).  Returns (theta float32 CUDA tensor, [(step, mean loss)])."""
    import torch
    k, T = data.k, data.T
    theta = torch.from_numpy(np.asarray(theta0, dtype=np.float32)).cuda()
    if theta.numel() != dmc.mlp_param_count(k):
        raise ValueError("theta0 has the wrong number of parameters for k")
    m = torch.zeros_like(theta)
    v = torch.zeros_like(theta)
    batch = min(batch, data.nb)
    nbatch = max(1, data.nb // batch)
    hist = []
    for step in range(1, steps + 1):
        b0 = ((step - 1) % nbatch) * batch
        S = data.S[b0:b0 + batch]
        U = data.U[b0:b0 + batch]
        Q, cache = dmc.mlp_forward(ctx, theta, k, S, cache=True)
        dQ, loss = dmc.mlp_loss_grad(ctx, Q.view(batch, T, k), U, mu)
        g = dmc.mlp_backward(ctx, theta, k, S, cache, dQ)
        dmc.mlp_adam(ctx, theta, g, m, v, step, lr)
        if step % log_every == 0 or step == steps:
            hist.append((step, float(loss.cpu().numpy().mean())))
    return theta, hist


def evaluate(ctx: dmc.Context, R_host: np.ndarray, theta, omega_host: np.ndarray, k: int, *,
             random_starts: np.ndarray, oi_tol: float = 1e-12, max_sweeps: int = 200):
    """Sweeps to tolerance and the largest principal angle (sine) between the
    start block and the converged subspace, for the learned start and for the
    plain Gaussian start, on held-out blocks [nb][T][T].  Returns a dict of
    per-block arrays."""
    import torch
    R = torch.from_numpy(np.ascontiguousarray(R_host, dtype=np.float64)).cuda()
    nb, T, _ = R_host.shape
    omega = torch.from_numpy(np.ascontiguousarray(omega_host, dtype=np.float64)).cuda()
    exact = dmc.make_params(k, precision=dmc.FP64, init=dmc.INIT_EXACT)
    U, _, _ = dmc.oi_blocks(ctx, R, exact)
    dmc.learned_start(ctx, T, k, omega, theta)
    try:
        pl = dmc.make_params(k, precision=dmc.FP64, init=dmc.INIT_LEARNED, oi_tol=oi_tol,
                             oi_max_sweeps=max_sweeps)
        _, sw_learned, res_learned = dmc.oi_blocks(ctx, R, pl)
        S = dmc.mlp_sketch(ctx, R, omega)
        Q0 = dmc.mlp_forward(ctx, theta, k, S).view(nb, T, k)
    finally:
        dmc.learned_start(ctx, 0, 0, None, None)
    qr = torch.from_numpy(np.ascontiguousarray(random_starts, dtype=np.float64)).cuda()
    pr = dmc.make_params(k, precision=dmc.FP64, init=dmc.INIT_RANDOM, oi_tol=oi_tol,
                         oi_max_sweeps=max_sweeps)
    _, sw_random, res_random = dmc.oi_blocks(ctx, R, pr, q_start=qr)
    Uh = U.cpu().numpy()
    Qh = Q0.cpu().numpy().astype(np.float64)
    return {"sweeps_learned": sw_learned, "sweeps_random": sw_random,
            "resid_learned": res_learned, "resid_random": res_random,
            "start_angle_learned": np.array([_sin_angle(Uh[b], Qh[b]) for b in range(nb)]),
            "start_angle_random": np.array([_sin_angle(Uh[b], random_starts[b]) for b in range(nb)]),
            "start_resid_learned": np.array([_start_resid(R_host[b], Qh[b]) for b in range(nb)]),
            "start_resid_random": np.array([_start_resid(R_host[b], random_starts[b])
                                            for b in range(nb)])}


def _sin_angle(U: np.ndarray, Q: np.ndarray) -> float:
    """Sine of the largest principal angle between span(U) (orthonormal) and
    span(Q) (any full-rank block): || (I - U U^T) orth(Q) ||_2 (host-side
    report of a result, not part of the path)."""
    Qo, _ = np.linalg.qr(Q)
    return float(np.linalg.norm(Qo - U @ (U.T @ Qo), 2))


def _start_resid(R: np.ndarray, Q: np.ndarray) -> float:
    """||R Q - Q Q^T R Q||_F / ||R||_F of orth(Q): how far the start already
    is from an invariant subspace (the quantity the tolerance test uses)."""
    Qo, _ = np.linalg.qr(Q)
    RQ = R @ Qo
    return float(np.linalg.norm(RQ - Qo @ (Qo.T @ RQ)) / np.linalg.norm(R))

