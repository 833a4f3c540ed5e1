"""Seeded inputs of the learned start: the sketch matrix Omega and initial
network weights.  Random draws only, no arithmetic of the method."""
from __future__ import annotations

import math

import numpy as np

SKETCH = 32   # columns of Omega
HIDDEN = 128  # hidden width


def sketch_omega(T: int, seed: int) -> np.ndarray:
    """Omega, a seeded standard Gaussian T x 32 block (float64)."""
    return np.random.default_rng(seed).standard_normal((T, SKETCH))


def mlp_init(k: int, seed: int) -> np.ndarray:
    """Flat float64 weights W1 [32][128], b1 [128], W2 [128][128], b2 [128],
    W3 [128][k], b3 [k] (row-major, in this order): weight matrices drawn
    N(0, 1 / fan_in), biases zero."""
    rng = np.random.default_rng(seed)
    parts = []
    for rows, cols in ((SKETCH, HIDDEN), (HIDDEN, HIDDEN), (HIDDEN, k)):
        parts.append(rng.standard_normal((rows, cols)).ravel() / math.sqrt(rows))
        parts.append(np.zeros(cols))
    return np.concatenate(parts)
