"""Float64 oracle of the learned warm start of the orthogonal iterations.

TEST INFRASTRUCTURE ONLY: imported by tests/, __graft_entry__.smoke() and
bench.py's CPU-baseline leg, never by the library.

The start block of a window's orthogonal iterations (Algorithm 1 takes any
orthonormal start) is predicted from a sketch of the window's autocorrelation
(Eq. 7): R Omega (Omega a fixed seeded Gaussian T x 32 block) with its
columns orthonormalised and scaled by sqrt(T), mapped row by row by a
three-layer perceptron
    h1 = gelu(S W1 + b1)      32 -> 128
    h2 = gelu(h1 W2 + b2)    128 -> 128
    Q  = h2 W3 + b3          128 -> k
with gelu(x) = x Phi(x) (Gaussian CDF, erf form).  The network is trained on
subspaces U_k the plain method converges to, with a loss that depends only on
span(Q) and on how far Q is from orthonormal:
    l(Q) = ||(I - U U^T) Q||_F^2 / ||Q||_F^2
           + mu || Q^T Q / (||Q||_F^2 / k) - I ||_F^2.
None of this is in the paper (it is the learned start the plain start falls
back to); everything here is float64 and written for checking, not speed.
"""
from __future__ import annotations

import math

import numpy as np

SKETCH = 32   # columns of Omega
HIDDEN = 128  # width of the two hidden layers


def param_shapes(k: int):
    """(name, shape) of every parameter, in storage order."""
    return [("W1", (SKETCH, HIDDEN)), ("b1", (HIDDEN,)), ("W2", (HIDDEN, HIDDEN)),
            ("b2", (HIDDEN,)), ("W3", (HIDDEN, k)), ("b3", (k,))]


def param_count(k: int) -> int:
    return sum(int(np.prod(s)) for _, s in param_shapes(k))


def unpack(theta: np.ndarray, k: int) -> dict:
    """Views of the flat parameter vector (storage order of param_shapes)."""
    out, o = {}, 0
    for name, shp in param_shapes(k):
        size = int(np.prod(shp))
        out[name] = theta[o:o + size].reshape(shp)
        o += size
    return out


def pack(p: dict, k: int) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel()
                           for name, _ in param_shapes(k)])


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round float32 values to the nearest bfloat16 (ties to even), returned
    as float64: keep the top 16 bits of the float32 encoding."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    b = f.view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    r = ((b + 0x7FFF + lsb) >> 16) << 16
    nan = np.isnan(f)
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    out[nan] = np.nan
    return out


SKETCH_DROP = 1e-10  # a sketch column with less than this fraction of its norm
                     # left after projection carries no direction: zeroed


def sketch(R: np.ndarray, omega: np.ndarray) -> np.ndarray:
    """Input rows of the network: the sketch R Omega with orthonormalised
    columns, scaled by sqrt(T) (entries of order one).  The columns of R Omega
    differ in size by the eigenvalue spread of R; orthonormalising exposes the
    smaller directions.  Classical Gram-Schmidt run twice per column, in
    column order; a column keeping less than SKETCH_DROP of its norm after the
    projections is set to zero (and projects nothing out of later columns)."""
    S = np.asarray(R, dtype=np.float64) @ np.asarray(omega, dtype=np.float64)
    T, m = S.shape
    Q = np.zeros_like(S)
    for j in range(m):
        v = S[:, j].copy()
        n0 = math.sqrt(float(v @ v))
        for _ in range(2):
            d = Q[:, :j].T @ v
            v = v - Q[:, :j] @ d
        nj = math.sqrt(float(v @ v))
        if n0 > 0.0 and nj > SKETCH_DROP * n0:
            Q[:, j] = v / nj
    return Q * math.sqrt(T)


def _Phi(x: np.ndarray) -> np.ndarray:
    """Standard normal CDF, 0.5 (1 + erf(x / sqrt 2)) written as
    0.5 erfc(-x / sqrt 2), which keeps its relative accuracy for x << 0."""
    erfc = np.vectorize(math.erfc)
    return 0.5 * erfc(-np.asarray(x, dtype=np.float64) / math.sqrt(2.0))


def gelu(x: np.ndarray) -> np.ndarray:
    """x Phi(x), Phi the standard normal CDF."""
    return x * _Phi(x)


def gelu_grad(x: np.ndarray) -> np.ndarray:
    """d/dx [x Phi(x)] = Phi(x) + x phi(x)."""
    Phi = _Phi(x)
    phi = np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)
    return Phi + x * phi


def forward(S: np.ndarray, theta: np.ndarray, k: int):
    """Rows of S (N x 32) -> Q (N x k); returns (Q, cache for backward)."""
    p = unpack(theta, k)
    z1 = S @ p["W1"] + p["b1"]
    h1 = gelu(z1)
    z2 = h1 @ p["W2"] + p["b2"]
    h2 = gelu(z2)
    Q = h2 @ p["W3"] + p["b3"]
    return Q, (S, z1, h1, z2, h2)


def backward(dQ: np.ndarray, theta: np.ndarray, k: int, cache) -> np.ndarray:
    """Gradient of sum(dQ * Q) with respect to every parameter (flat, in
    storage order), by the chain rule through the three layers."""
    S, z1, h1, z2, h2 = cache
    p = unpack(theta, k)
    g = {}
    g["W3"] = h2.T @ dQ
    g["b3"] = dQ.sum(axis=0)
    dz2 = (dQ @ p["W3"].T) * gelu_grad(z2)
    g["W2"] = h1.T @ dz2
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2 @ p["W2"].T) * gelu_grad(z1)
    g["W1"] = S.T @ dz1
    g["b1"] = dz1.sum(axis=0)
    return pack(g, k)


def subspace_loss(Q: np.ndarray, U: np.ndarray, mu: float = 0.1):
    """Loss of one T x k start block Q against the orthonormal target U and its
    gradient dl/dQ:
      term 1 = ||(I - U U^T) Q||^2 / ||Q||^2 = 1 - ||U^T Q||^2 / n2,
      term 2 = mu ||c G - I||^2 with G = Q^T Q, n2 = trace G, c = k / n2."""
    Q = np.asarray(Q, dtype=np.float64)
    U = np.asarray(U, dtype=np.float64)
    k = Q.shape[1]
    G = Q.T @ Q
    n2 = float(np.trace(G))
    A = U.T @ Q
    a2 = float(np.sum(A * A))
    c = k / n2
    M = c * G - np.eye(k)
    loss = (1.0 - a2 / n2) + mu * float(np.sum(M * M))
    mg = float(np.sum(M * G))
    grad = (-2.0 / n2) * (U @ A) + (2.0 * a2 / n2 ** 2) * Q \
        + mu * (4.0 * c * (Q @ M) - (4.0 * k * mg / n2 ** 2) * Q)
    return loss, grad


def batch_loss(Qs: np.ndarray, Us: np.ndarray, mu: float = 0.1):
    """Mean of subspace_loss over blocks [nb][T][k]; gradient of the mean."""
    nb = Qs.shape[0]
    tot, grads = 0.0, np.empty_like(np.asarray(Qs, dtype=np.float64))
    for b in range(nb):
        l, g = subspace_loss(Qs[b], Us[b], mu)
        tot += l
        grads[b] = g / nb
    return tot / nb, grads


def predict_start(R: np.ndarray, omega: np.ndarray, theta: np.ndarray, k: int) -> np.ndarray:
    """The learned start block of one coordinate's window: MLP(sketch(R))."""
    Q, _ = forward(sketch(R, omega), theta, k)
    return Q


def adam_step(theta, grad, m, v, step: int, lr: float, b1: float = 0.9, b2: float = 0.999,
              eps: float = 1e-8):
    """One Adam update (Kingma and Ba), bias-corrected; returns new arrays."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
