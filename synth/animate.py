"""Seeded synthetic animations of a fixed-connectivity mesh, plus the other
random inputs the compressor takes (anchor index sets, a Gaussian initial
subspace).

All draws come from ``numpy.random.default_rng(seed)`` in a fixed order, so the
same seed gives the same frames on every machine.  Frames are returned as
``[F][n][3]`` (frame-major, xyz interleaved), the layout the compressor reads.
"""
from __future__ import annotations

import numpy as np


def _unit(v):
    return v / np.linalg.norm(v)


def _random_axis(rng):
    return _unit(rng.standard_normal(3))


def _rodrigues(axis, angle):
    """Rotation matrices for angle[...] about one unit axis: [..., 3, 3]."""
    kx, ky, kz = axis
    K = np.array([[0.0, -kz, ky], [kz, 0.0, -kx], [-ky, kx, 0.0]])
    a = np.asarray(angle, dtype=np.float64)[..., None, None]
    return np.eye(3) + np.sin(a) * K + (1.0 - np.cos(a)) * (K @ K)


def bend_twist(rest, n_frames: int, seed: int, amplitude: float = 0.2,
               period_range=(8.0, 32.0), noise_var: float = 1e-4,
               dtype=np.float64):
    """Three smooth sinusoidal deformation fields applied in order, then i.i.d.
    Gaussian noise of variance `noise_var` on every coordinate.

    Field f has a unit axis a_f, period P_f ~ U[period_range], phase
    phi_f ~ U[0, 2pi) and strength s_f(t) = amplitude * sin(2 pi t / P_f + phi_f).
    Fields 0 and 2 twist (rotate p about a_f by s_f(t) * (a_f . p));
    field 1 bends (p += s_f(t) * (a_f . p)^2 * b_f, with b_f a unit vector
    orthogonal to a_f).
    """
    rng = np.random.default_rng(seed)
    fields = []
    for f in range(3):
        a = _random_axis(rng)
        period = rng.uniform(*period_range)
        phase = rng.uniform(0.0, 2.0 * np.pi)
        bdir = None
        if f == 1:
            r = rng.standard_normal(3)
            bdir = _unit(r - np.dot(r, a) * a)
        fields.append((a, period, phase, bdir))
    t = np.arange(n_frames, dtype=np.float64)
    P = np.broadcast_to(rest, (n_frames,) + rest.shape).copy()
    for f, (a, period, phase, bdir) in enumerate(fields):
        s = amplitude * np.sin(2.0 * np.pi * t / period + phase)  # [F]
        proj = P @ a  # [F][n]
        if bdir is None:
            ang = s[:, None] * proj  # [F][n]
            # Rodrigues per point: p cos + (a x p) sin + a (a.p)(1 - cos)
            c, sn = np.cos(ang)[..., None], np.sin(ang)[..., None]
            cross = np.cross(np.broadcast_to(a, P.shape), P)
            P = P * c + cross * sn + a * (proj[..., None] * (1.0 - c))
        else:
            P = P + (s[:, None] * proj * proj)[..., None] * bdir
    noise = rng.standard_normal(P.shape) * np.sqrt(noise_var)
    return (P + noise).astype(dtype)


def _rbf_rig(rest, n_bones: int, seed: int, max_angle_deg: float, period_range,
             root_weight: float, sigma_frac: float):
    """The seeded bones (centre, axis, theta_max, period, phase) and the
    normalised weights [n][n_bones + 1] of rbf_skinning."""
    rng = np.random.default_rng(seed)
    n = rest.shape[0]
    bones = []
    for _ in range(n_bones):
        centre = rest[rng.integers(0, n)].copy()
        axis = _random_axis(rng)
        theta_max = np.deg2rad(max_angle_deg) * (1.0 - rng.uniform(0.0, 1.0))
        period = rng.uniform(*period_range)
        phase = rng.uniform(0.0, 2.0 * np.pi)
        bones.append((centre, axis, theta_max, period, phase))
    diag = np.linalg.norm(rest.max(axis=0) - rest.min(axis=0))
    sigma = sigma_frac * diag
    W = np.empty((n, n_bones + 1))
    for b, (c, *_rest) in enumerate(bones):
        d2 = np.sum((rest - c) ** 2, axis=1)
        W[:, b] = np.exp(-d2 / (2.0 * sigma * sigma))
    W[:, n_bones] = root_weight
    W /= W.sum(axis=1, keepdims=True)
    return bones, W


def rbf_skinning_torch(rest, n_frames: int, n_bones: int, seed: int, device,
                       max_angle_deg: float = 30.0, period_range=(16.0, 128.0),
                       root_weight: float = 0.1, sigma_frac: float = 0.25, t0: int = 0,
                       frames_per_chunk: int = 32):
    """rbf_skinning with the same seeded rig, evaluated with torch (float64)
    on `device` and returned there as float32 [n_frames][n][3]: for the large
    training sets of the learned start (input synthesis only)."""
    import torch
    bones, W = _rbf_rig(rest, n_bones, seed, max_angle_deg, period_range, root_weight, sigma_frac)
    n = rest.shape[0]
    P = torch.from_numpy(np.asarray(rest, dtype=np.float64)).to(device)
    Wt = torch.from_numpy(W).to(device)
    t = t0 + np.arange(n_frames, dtype=np.float64)
    rots = [torch.from_numpy(_rodrigues(axis, theta_max * np.sin(2.0 * np.pi * t / period + phase)))
            .to(device) for (c, axis, theta_max, period, phase) in bones]
    centres = [torch.from_numpy(np.asarray(c, dtype=np.float64)).to(device) for (c, *_r) in bones]
    out = torch.empty((n_frames, n, 3), dtype=torch.float32, device=device)
    for f0 in range(0, n_frames, frames_per_chunk):
        f1 = min(n_frames, f0 + frames_per_chunk)
        acc = (Wt[:, n_bones:n_bones + 1] * P).unsqueeze(0).repeat(f1 - f0, 1, 1)
        for b in range(n_bones):
            rel = P - centres[b]
            moved = torch.matmul(rel.unsqueeze(0), rots[b][f0:f1].transpose(1, 2).contiguous())
            acc += Wt[:, b:b + 1].unsqueeze(0) * (moved + centres[b])
        out[f0:f1] = acc.to(torch.float32)
    return out


def rbf_skinning(rest, n_frames: int, n_bones: int, seed: int,
                 max_angle_deg: float = 30.0, period_range=(16.0, 128.0),
                 root_weight: float = 0.1, sigma_frac: float = 0.25,
                 t0: int = 0, dtype=np.float32):
    """Gaussian-RBF skinning with `n_bones` bones rotating sinusoidally.

    Bone b: centre c_b = a random rest vertex, axis uniform on the sphere,
    angle theta_b(t) = theta_max_b * sin(2 pi t / P_b + phi_b) with
    theta_max_b ~ U(0, max_angle], P_b ~ U[period_range], phi_b ~ U[0, 2pi).
    Weights w_b(p) = exp(-|p - c_b|^2 / (2 sigma^2)), sigma = sigma_frac times
    the bounding-box diagonal, plus a static root weight, normalised per vertex.
    p(t) = sum_b w_b (R_b(t)(p - c_b) + c_b) + w_root p, t = t0 + frame index.
    """
    n = rest.shape[0]
    bones, W = _rbf_rig(rest, n_bones, seed, max_angle_deg, period_range, root_weight, sigma_frac)
    out = np.empty((n_frames, n, 3), dtype=dtype)
    t = t0 + np.arange(n_frames, dtype=np.float64)
    rots = []
    for (c, axis, theta_max, period, phase) in bones:
        ang = theta_max * np.sin(2.0 * np.pi * t / period + phase)
        rots.append(_rodrigues(axis, ang))  # [F][3][3]
    for f in range(n_frames):
        acc = W[:, n_bones:n_bones + 1] * rest
        for b, (c, *_r) in enumerate(bones):
            acc += W[:, b:b + 1] * ((rest - c) @ rots[b][f].T + c)
        out[f] = acc
    return out


def choose_anchors(n: int, n_anchors: int, seed: int) -> np.ndarray:
    """Seeded uniform sample of distinct vertex indices, sorted (int32)."""
    if not 0 < n_anchors <= n:
        raise ValueError("need 0 < n_anchors <= n")
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n, n_anchors, replace=False)).astype(np.int32)


def default_anchor_count(n: int) -> int:
    """One per cent of the vertices, at least one."""
    return max(1, int(round(0.01 * n)))


def gaussian_subspace(T: int, k: int, seed: int) -> np.ndarray:
    """A seeded Gaussian T x k block per coordinate: [3][T][k] float64.

    Used as the starting block of orthogonal iterations when no previous
    window and no exact start is wanted.
    """
    rng = np.random.default_rng(seed)
    return rng.standard_normal((3, T, k))


def gapped_windows(rest, n_frames: int, T: int, k: int, seed: int, gap: float = 4.0,
                   decay: float = 0.1, scale: float = 0.1, drift=None, dtype=np.float64):
    """Frames whose every window of T frames has, per coordinate, an
    autocorrelation with a clean eigenvalue gap after its k-th eigenvalue.

    The T x n matrix of a window's coordinate c is A_c = U (S V^T + sqrt(T)
    e_0 r_c^T), with r_c the rest pose's coordinate c, U (T x T) a seeded
    orthonormal block whose first column is constant (1/sqrt(T)), V (n x T)
    seeded orthonormal columns orthogonal to r_c, and S = diag(s) scaled by
    scale sqrt(n): s_j = 2^(-decay j) for j < k and
    s_(k-1) 2^(-decay (j - k + 1)) / gap beyond.  Then A_c A_c^T =
    U diag(s_0^2 + T |r_c|^2, s_1^2, ...) U^T exactly: frame t is the rest
    pose plus a deformation, lambda_k / lambda_(k+1) is about gap^2, and the
    trailing eigenvalues stay far above round-off.  A shorter last window uses
    its own length T_w and k_w = min(k, T_w).  With `drift`, the full windows
    share one seeded U per coordinate, perturbed per window by drift times a
    Gaussian block before orthonormalisation, so consecutive windows have
    nearby eigenvectors."""
    rng = np.random.default_rng(seed)
    n = rest.shape[0]
    out = np.empty((n_frames, n, 3), dtype=np.float64)
    base = [rng.standard_normal((T, T)) for _ in range(3)] if drift is not None else None
    for s0 in range(0, n_frames, T):
        tw = min(T, n_frames - s0)
        kw = min(k, tw)
        j = np.arange(tw, dtype=np.float64)
        s = np.where(j < kw, 2.0 ** (-decay * j),
                     2.0 ** (-decay * (kw - 1)) * 2.0 ** (-decay * (j - kw + 1)) / gap)
        s = s * scale * np.sqrt(n)
        for c in range(3):
            if base is not None and tw == T:
                G = base[c] + drift * rng.standard_normal((tw, tw))
            else:
                G = rng.standard_normal((tw, tw))
            G[:, 0] = 1.0
            U, _ = np.linalg.qr(G)
            U[:, 0] = np.abs(U[:, 0])  # the constant column, positive
            r = rest[:, c].astype(np.float64)
            B = rng.standard_normal((n, tw + 1))
            B[:, 0] = r
            Qb, _ = np.linalg.qr(B)
            V = Qb[:, 1:]  # orthonormal, orthogonal to r
            out[s0:s0 + tw, :, c] = (U * s) @ V.T + np.outer(U[:, 0] * np.sqrt(tw), r)
    return out.astype(dtype)
