"""The named synthetic workloads, with their sizes and seeds.

  plain_fp64  : icosphere level 3 (642 vertices), 32 frames, three bend/twist
                fields + noise, one 32-frame window, k = 8, 12-bit codes,
                8 anchors, float64.
  torus_fp32  : 128 x 128 torus (16,384 vertices), 256 frames in 32-frame
                windows (8 windows), 6-bone RBF skinning, k = 16, 12-bit
                codes, 64 anchors, float32.
  icosphere7  : icosphere level 7 (163,842 vertices), 512 frames in 64-frame
                windows, 8-bone RBF skinning, k = 32, 10-bit codes, 1,638
                anchors.

Each entry builds a `Workload` (frames, mesh, anchors, parameters) from its
seeds alone.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import animate, meshes


@dataclass
class Workload:
    name: str
    verts: np.ndarray          # rest pose [n][3] float64
    tris: np.ndarray           # [n_tris][3] int32
    frames: np.ndarray         # [F][n][3] float32 or float64
    anchors: np.ndarray        # sorted int32 [n_c]
    T: int                     # window length (frames)
    k: int                     # retained rows per window
    bits: int                  # coefficient quantiser bits (0 = raw)
    precision: str             # "fp64" | "fp32"
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.verts.shape[0]

    @property
    def F(self) -> int:
        return self.frames.shape[0]


def plain_fp64() -> Workload:
    v, t = meshes.icosphere(3)
    fr = animate.bend_twist(v, 32, seed=101, dtype=np.float64)
    anc = animate.choose_anchors(v.shape[0], 8, seed=102)
    return Workload("icosphere3-642v-32f-T32-k8-b12-fp64", v, t, fr, anc,
                    T=32, k=8, bits=12, precision="fp64")


def torus_fp32(frames: int = 256) -> Workload:
    v, t = meshes.torus(128, 128)
    fr = animate.rbf_skinning(v, frames, 6, seed=202, dtype=np.float32)
    anc = animate.choose_anchors(v.shape[0], 64, seed=203)
    return Workload("torus128x128-16384v-256f-T32-k16-b12-fp32", v, t, fr, anc,
                    T=32, k=16, bits=12, precision="fp32")


def icosphere7(frames: int = 512) -> Workload:
    v, t = meshes.icosphere(7)
    fr = animate.rbf_skinning(v, frames, 8, seed=303, dtype=np.float32)
    anc = animate.choose_anchors(v.shape[0], 1638, seed=304)
    return Workload("icosphere7-163842v-512f-T64-k32-b10", v, t, fr, anc,
                    T=64, k=32, bits=10, precision="fp32")


def small_torus(a: int = 24, b: int = 20, frames: int = 40, T: int = 16, k: int = 6,
                bits: int = 12, n_anchors: int = 6, seed: int = 11,
                precision: str = "fp64") -> Workload:
    """A small torus animation for fast tests (ragged last window by default)."""
    v, t = meshes.torus(a, b)
    dt = np.float64 if precision == "fp64" else np.float32
    fr = animate.rbf_skinning(v, frames, 4, seed=seed, dtype=dt)
    anc = animate.choose_anchors(v.shape[0], n_anchors, seed=seed + 1)
    return Workload(f"torus{a}x{b}-{frames}f-T{T}-k{k}", v, t, fr, anc,
                    T=T, k=k, bits=bits, precision=precision)


def batched(count: int = 64, n_range=(2000, 60000), f_range=(16, 128), ks=(8, 16, 32),
            seed: int = 4000, bones: int = 6, only=None):
    """Independent sequences of uneven size for the batched form: mesh type
    torus or icosphere (the icosphere level whose size is nearest the drawn
    n, from levels 2..6), torus a = round(sqrt(n)), b = round(n / a); frame
    count uniform in f_range, k drawn from ks, window T = 2k, 1% anchors (at
    least 4), RBF skinning seeded per sequence, float32.  `only`: indices of
    the sequences to build (the draws of the others are still made, so each
    sequence is the same as in the full batch)."""
    rng = np.random.default_rng(seed)
    out = []
    levels = {L: 10 * 4 ** L + 2 for L in range(2, 7)}
    for i in range(count):
        n_target = int(rng.integers(n_range[0], n_range[1] + 1))
        if rng.random() < 0.5:
            a = max(3, int(round(np.sqrt(n_target))))
            b = max(3, int(round(n_target / a)))
            v, t = meshes.torus(a, b)
            name = f"torus{a}x{b}"
        else:
            L = min(levels, key=lambda x: abs(levels[x] - n_target))
            v, t = meshes.icosphere(L)
            name = f"icosphere{L}"
        F = int(rng.integers(f_range[0], f_range[1] + 1))
        k = int(ks[int(rng.integers(0, len(ks)))])
        if only is not None and i not in only:
            continue
        fr = animate.rbf_skinning(v, F, bones, seed=seed + 1 + i, dtype=np.float32)
        nc = max(4, int(round(0.01 * v.shape[0])))
        anc = animate.choose_anchors(v.shape[0], nc, seed=seed + 1001 + i)
        out.append(Workload(f"{name}-{F}f-T{2 * k}-k{k}", v, t, fr, anc, T=2 * k, k=k, bits=12,
                            precision="fp32"))
    return out


REGISTRY = {
    "plain_fp64": plain_fp64,
    "torus_fp32": torus_fp32,
    "icosphere7": icosphere7,
}
