"""Pins of the learned-start oracle (oracle/mlp_oracle.py): library routines,
finite differences, closed forms and invariances.  CPU only."""
import math

import numpy as np
import pytest

from oracle import mlp_oracle as M
from synth import learned


def test_gelu_matches_normal_cdf():
    from scipy.stats import norm
    x = np.linspace(-9, 9, 181)
    np.testing.assert_allclose(M.gelu(x), x * norm.cdf(x), rtol=1e-13, atol=1e-300)
    assert M.gelu(np.array([0.0]))[0] == 0.0


def test_gelu_grad_central_differences():
    x = np.linspace(-6, 6, 97)
    h = 1e-6
    fd = (M.gelu(x + h) - M.gelu(x - h)) / (2 * h)
    np.testing.assert_allclose(M.gelu_grad(x), fd, rtol=1e-7, atol=1e-9)


def test_bf16_round_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(5000) * 10.0 ** rng.integers(-30, 30, 5000),
                        [1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -1.0 - 2 ** -8, 0.0, -0.0,
                         3.0e38, 1e-40]]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(M.bf16_round(x), ref)
    # ties go to the even neighbour
    assert M.bf16_round(np.array([1.0 + 2 ** -8]))[0] == 1.0
    assert M.bf16_round(np.array([1.0 + 3 * 2 ** -8]))[0] == 1.0 + 2 ** -6


def test_sketch_is_scaled_q_factor_of_r_omega():
    """On a well-conditioned sketch the features are sqrt(T) times LAPACK's Q
    factor of R Omega (positive diagonal); scaling R changes nothing."""
    rng = np.random.default_rng(1)
    A = rng.standard_normal((40, 300))
    R = A @ A.T
    om = rng.standard_normal((40, M.SKETCH))
    S = M.sketch(R, om)
    Qr, Rr = np.linalg.qr(R @ om)
    Qr = Qr * np.sign(np.diag(Rr))
    np.testing.assert_allclose(S, math.sqrt(40) * Qr, atol=1e-10)
    np.testing.assert_allclose(S.T @ S / 40, np.eye(M.SKETCH), atol=1e-12)
    np.testing.assert_allclose(M.sketch(7.5 * R, om), S, atol=1e-12)


def test_sketch_drops_directions_without_content():
    """A rank-5 R: the first five columns span range(R), the others are zero."""
    rng = np.random.default_rng(2)
    B = rng.standard_normal((24, 5))
    R = B @ B.T
    S = M.sketch(R, rng.standard_normal((24, M.SKETCH)))
    assert np.all(np.linalg.norm(S[:, 5:], axis=0) == 0.0)
    P = B @ np.linalg.pinv(B)
    np.testing.assert_allclose(P @ S[:, :5], S[:, :5], atol=1e-10)


@pytest.mark.parametrize("k", [4, 16, 32])
def test_backward_central_differences(k):
    rng = np.random.default_rng(k)
    theta = learned.mlp_init(k, seed=k) + 0.05 * rng.standard_normal(M.param_count(k))
    S = rng.standard_normal((9, M.SKETCH))
    dQ = rng.standard_normal((9, k))
    Q, cache = M.forward(S, theta, k)
    g = M.backward(dQ, theta, k, cache)
    idx = rng.choice(theta.size, 60, replace=False)
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (np.sum(dQ * M.forward(S, tp, k)[0]) - np.sum(dQ * M.forward(S, tm, k)[0])) / (2 * h)
        assert abs(g[i] - fd) <= 1e-6 * max(1.0, abs(fd)), (i, g[i], fd)


def test_loss_gradient_central_differences():
    rng = np.random.default_rng(2)
    T, k = 12, 5
    U = np.linalg.qr(rng.standard_normal((T, k)))[0]
    Q = rng.standard_normal((T, k))
    l0, g = M.subspace_loss(Q, U, 0.1)
    h = 1e-6
    for i in range(T):
        for j in range(k):
            Qp, Qm = Q.copy(), Q.copy()
            Qp[i, j] += h
            Qm[i, j] -= h
            fd = (M.subspace_loss(Qp, U, 0.1)[0] - M.subspace_loss(Qm, U, 0.1)[0]) / (2 * h)
            assert abs(g[i, j] - fd) <= 1e-7 * max(1.0, abs(fd))


def test_loss_zero_on_target_and_invariant():
    rng = np.random.default_rng(3)
    T, k = 16, 6
    U = np.linalg.qr(rng.standard_normal((T, k)))[0]
    assert abs(M.subspace_loss(U, U)[0]) < 1e-14
    G = np.linalg.qr(rng.standard_normal((k, k)))[0]
    assert abs(M.subspace_loss(3.7 * U @ G, U)[0]) < 1e-13      # rotation + scale
    Q = rng.standard_normal((T, k))
    l1 = M.subspace_loss(Q, U)[0]
    l2 = M.subspace_loss(0.01 * Q @ G, U)[0]
    assert abs(l1 - l2) < 1e-12
    # first term alone lies in [0, 1]: 0 inside span(U), 1 orthogonal to it
    P = np.eye(T) - U @ U.T
    W = P @ rng.standard_normal((T, k))
    W = np.linalg.qr(W)[0]
    assert abs(M.subspace_loss(W, U, mu=0.0)[0] - 1.0) < 1e-13


def test_adam_first_step_is_signed_learning_rate():
    rng = np.random.default_rng(4)
    th = rng.standard_normal(50)
    g = rng.standard_normal(50)
    new, m, v = M.adam_step(th, g, np.zeros(50), np.zeros(50), step=1, lr=1e-3, eps=0.0)
    np.testing.assert_allclose(new, th - 1e-3 * np.sign(g), rtol=0, atol=1e-15)


def test_param_count_and_layout():
    assert M.param_count(32) == 24864
    th = np.arange(M.param_count(8), dtype=np.float64)
    p = M.unpack(th, 8)
    assert p["W1"].shape == (32, 128) and p["b3"].shape == (8,)
    np.testing.assert_array_equal(M.pack(p, 8), th)


def test_generator_layout_matches_oracle():
    th = learned.mlp_init(16, seed=1)
    assert th.size == M.param_count(16)
    p = M.unpack(th, 16)
    assert np.all(p["b1"] == 0) and np.all(p["b3"] == 0)
    assert abs(np.std(p["W2"]) * math.sqrt(128) - 1.0) < 0.05
    assert learned.sketch_omega(64, 3).shape == (64, M.SKETCH)
