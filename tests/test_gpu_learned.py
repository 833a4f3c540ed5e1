"""The learned start on the GPU (through the C ABI) against the float64 oracle
of oracle/mlp_oracle.py: sketch, forward, loss, backward and Adam kernels,
orthogonal iterations on independent blocks, training on the GPU and what the
trained network gains over the plain start on held-out animations."""
import numpy as np
import pytest

import oracle as O
from oracle import mlp_oracle as M
from paper_2111_10105_amd import dmc, learned as L
from synth import animate, configs, learned, meshes

from gpu_helpers import sin_angle, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(gpu):
    c = dmc.Context(0)
    yield c
    c.close()


def _np(t):
    return t.detach().cpu().numpy()


def _theta(k, seed):
    """Seeded weights with non-zero biases."""
    rng = np.random.default_rng(seed + 1000)
    return learned.mlp_init(k, seed) + 0.05 * rng.standard_normal(M.param_count(k))


def _effective(theta32, k):
    """The parameters the GPU computes with: weight matrices rounded to
    bfloat16, biases float32."""
    p = M.unpack(np.asarray(theta32, dtype=np.float64), k)
    for name in ("W1", "W2", "W3"):
        p[name] = M.bf16_round(p[name])
    return M.pack(p, k)


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def _cos(a, b):
    a, b = np.ravel(a), np.ravel(b)
    return float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b)))


def _spd_blocks(nb, T, seed, rank=None):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(nb):
        A = rng.standard_normal((T, rank or 3 * T)) * np.logspace(0, -3, rank or 3 * T)
        out.append(A @ A.T)
    return np.stack(out)


def test_mlp_sketch_matches_oracle(ctx):
    T = 40
    R = _spd_blocks(5, T, 1)
    om = learned.sketch_omega(T, 2)
    S = _np(dmc.mlp_sketch(ctx, to_dev(R), to_dev(om)))
    for b in range(5):
        ref = M.sketch(R[b], om)
        assert np.max(np.abs(S[b] - ref)) <= 1e-6 * np.abs(ref).max()


@pytest.mark.parametrize("k", [8, 16, 32])
def test_mlp_forward_matches_oracle(ctx, k):
    """150 rows (a ragged last tile of the 64-row kernel)."""
    theta = _theta(k, k).astype(np.float32)
    S = np.random.default_rng(k).standard_normal((150, 32)).astype(np.float32)
    Q = _np(dmc.mlp_forward(ctx, to_dev(theta), k, to_dev(S)))
    ref, _ = M.forward(M.bf16_round(S), _effective(theta, k), k)
    assert _rel(Q, ref) <= 1e-2 and _cos(Q, ref) > 0.999, (_rel(Q, ref), _cos(Q, ref))


def test_mlp_loss_grad_matches_oracle(ctx):
    nb, T, k = 6, 48, 20
    rng = np.random.default_rng(7)
    Q = rng.standard_normal((nb, T, k)).astype(np.float32)
    U = np.stack([np.linalg.qr(rng.standard_normal((T, k)))[0] for _ in range(nb)])
    dQ, loss = dmc.mlp_loss_grad(ctx, to_dev(Q), to_dev(U), 0.1)
    ref_l = [M.subspace_loss(Q[b].astype(np.float64), U[b], 0.1)[0] for b in range(nb)]
    _, ref_g = M.batch_loss(Q.astype(np.float64), U, 0.1)
    np.testing.assert_allclose(_np(loss), ref_l, rtol=1e-5)
    assert _rel(_np(dQ), ref_g) <= 1e-4


@pytest.mark.parametrize("k", [8, 32])
def test_mlp_backward_matches_oracle(ctx, k):
    """Gradients of every parameter tensor against the float64 oracle on the
    bfloat16-rounded weights: relative error <= 1e-2, cosine > 0.999."""
    theta = _theta(k, 3 + k).astype(np.float32)
    rng = np.random.default_rng(11 + k)
    N = 333
    S = rng.standard_normal((N, 32)).astype(np.float32)
    dQ = rng.standard_normal((N, k)).astype(np.float32)
    th = to_dev(theta)
    Q, cache = dmc.mlp_forward(ctx, th, k, to_dev(S), cache=True)
    g = _np(dmc.mlp_backward(ctx, th, k, to_dev(S), cache, to_dev(dQ)))
    eff = _effective(theta, k)
    _, c = M.forward(M.bf16_round(S), eff, k)
    ref = M.backward(dQ.astype(np.float64), eff, k, c)
    gp, rp = M.unpack(g.astype(np.float64), k), M.unpack(ref, k)
    for name, _ in M.param_shapes(k):
        r, cs = _rel(gp[name], rp[name]), _cos(gp[name], rp[name])
        print(f"grad {name}: rel {r:.2e} cos {cs:.6f}")
        assert r <= 1e-2 and cs > 0.999, name


def test_mlp_adam_matches_oracle(ctx):
    import torch
    rng = np.random.default_rng(5)
    n = 5000
    th, g = rng.standard_normal(n).astype(np.float32), rng.standard_normal(n).astype(np.float32)
    m0, v0 = (0.1 * rng.standard_normal(n)).astype(np.float32), rng.random(n).astype(np.float32)
    t, m, v = to_dev(th), to_dev(m0), to_dev(v0)
    dmc.mlp_adam(ctx, t, to_dev(g), m, v, step=7, lr=1e-3)
    torch.cuda.synchronize()
    ref, rm, rv = M.adam_step(th.astype(np.float64), g.astype(np.float64), m0.astype(np.float64),
                              v0.astype(np.float64), 7, 1e-3)
    np.testing.assert_allclose(_np(t), ref, rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(_np(m), rm, rtol=1e-5, atol=2e-7)


@pytest.mark.parametrize("init", [dmc.INIT_EXACT, dmc.INIT_RANDOM, dmc.INIT_SKETCH])
def test_oi_blocks_reach_jacobi_subspace(ctx, init):
    """Independent gapped blocks, every start: largest principal angle to the
    oracle's Jacobi eigenvectors < 1e-10, Q^T Q = I."""
    T, k, nb = 24, 5, 7
    rng = np.random.default_rng(9)
    R = []
    for _ in range(nb):
        V = np.linalg.qr(rng.standard_normal((T, T)))[0]
        lam = np.concatenate([np.logspace(2, 1, k), np.logspace(-1, -4, T - k)])
        R.append((V * lam) @ V.T)
    R = np.stack(R)
    p = dmc.make_params(k, precision=dmc.FP64, init=init, oi_tol=1e-14, oi_max_sweeps=500)
    q = {dmc.INIT_EXACT: None, dmc.INIT_RANDOM: rng.standard_normal((nb, T, k)),
         dmc.INIT_SKETCH: rng.standard_normal((T, k))}[init]
    U, sweeps, resid = dmc.oi_blocks(ctx, to_dev(R), p, q_start=None if q is None else to_dev(q))
    U = _np(U)
    for b in range(nb):
        _, V = O.jacobi_eigh(R[b])
        assert np.max(np.abs(U[b].T @ U[b] - np.eye(k))) < 1e-13
        assert sin_angle(V[:, :k], U[b]) < 1e-10
    if init == dmc.INIT_EXACT:
        assert np.all(sweeps == 0)
    else:
        assert np.all(sweeps >= 1) and np.all(resid <= 1e-14)


def _animation_blocks(seeds, T, F, n_bones=(8, 16)):
    """Autocorrelation blocks [3 * windows][T][T] of seeded RBF animations on
    small tori and icospheres (the oracle computes R, Eq. 7)."""
    out = []
    for s in seeds:
        rng = np.random.default_rng(s)
        if s % 2:
            v, _ = meshes.torus(int(rng.integers(30, 50)), int(rng.integers(30, 50)))
        else:
            v, _ = meshes.icosphere(4)
        fr = animate.rbf_skinning(v, F, int(rng.integers(n_bones[0], n_bones[1] + 1)), seed=s)
        for w0 in range(0, F, T):
            for c in range(3):
                out.append(O.autocorrelation(O.coordinate_matrix(fr[w0:w0 + T], c)))
    return np.stack(out)


def test_learned_start_trains_on_gpu_and_helps_on_held_out(ctx):
    """Train the network on the GPU on subspaces of seeded animations, then
    compare it with the plain Gaussian start on held-out animations at equal
    tolerance: the learned start begins closer to an invariant subspace and
    needs no more sweeps."""
    T, k = 64, 32
    train_R = _animation_blocks(range(5000, 5012), T, 256)
    test_R = _animation_blocks(range(7000, 7003), T, 128)
    perm = np.random.default_rng(0).permutation(train_R.shape[0])
    om = learned.sketch_omega(T, 4242)
    data = L.Dataset(ctx, train_R[perm], om, k)
    theta, hist = L.train(ctx, data, learned.mlp_init(k, 17), steps=600, batch=24, lr=2e-3)
    print("loss history", hist)
    assert hist[-1][1] < hist[0][1]
    rs = np.stack([animate.gaussian_subspace(T, k, 900 + b)[0] for b in range(test_R.shape[0])])
    ev = L.evaluate(ctx, test_R, theta, om, k, random_starts=rs)
    for key, v in ev.items():
        print(key, np.round(np.mean(v), 6), np.round(np.max(v), 6))
    assert np.mean(ev["start_resid_learned"]) < 0.5 * np.mean(ev["start_resid_random"])
    assert np.sum(ev["sweeps_learned"]) <= np.sum(ev["sweeps_random"])
    assert np.all(ev["resid_learned"] <= 1e-12) and np.all(ev["resid_random"] <= 1e-12)


@pytest.mark.parametrize("prec", [dmc.FP64, dmc.FP32])
def test_sequence_with_learned_start(ctx, prec):
    """compress_sequence with the learned start against the oracle given the
    same network (its float64 forward on the bfloat16-rounded weights)."""
    w = configs.small_torus(frames=56, T=16, k=10, precision="fp64" if prec == dmc.FP64 else "fp32")
    m = dmc.Mesh(ctx, w.n, w.tris, w.anchors)
    theta = _theta(w.k, 31).astype(np.float32)
    om = learned.sketch_omega(w.T, 77)
    dmc.learned_start(ctx, w.T, w.k, to_dev(om), to_dev(theta))
    try:
        p = dmc.make_params(w.k, coef_bits=w.bits, precision=prec, cg_tol=1e-13,
                            init=dmc.INIT_LEARNED)
        codes, out, stats, status = dmc.compress_sequence(ctx, m, to_dev(w.frames), w.T, p)
    finally:
        dmc.learned_start(ctx, 0, 0, None, None)
    assert status == 0
    sweeps = [s["oi_sweeps"] for s in stats]
    assert all(min(s) >= 1 for s in sweeps[:3]) and sweeps[3] == [0, 0, 0]
    _, ref = O.compress_sequence(w.n, w.tris, w.frames, w.anchors, w.T, w.k, w.bits, init="learned",
                                 learned=(om, _effective(theta, w.k)), fp32_data=(prec == dmc.FP32))
    got = _np(out)
    e_or, e_in, r_in = O.nmse(got, ref), O.nmse(got, w.frames), O.nmse(ref, w.frames)
    print(f"learned {prec}: sweeps {sweeps} NMSE(gpu,oracle)={e_or:.3e} NMSE(gpu,input)={e_in:.3e} "
          f"NMSE(oracle,input)={r_in:.3e}")
    assert e_or <= 0.5 * r_in
    assert e_in <= 1.1 * r_in


def test_learned_start_errors(ctx):
    w = configs.small_torus(frames=32, T=16, k=10, precision="fp32")
    m = dmc.Mesh(ctx, w.n, w.tris, w.anchors)
    p = dmc.make_params(w.k, coef_bits=w.bits, precision=dmc.FP32, init=dmc.INIT_LEARNED)
    with pytest.raises(dmc.DmcError):  # no network registered
        dmc.compress_sequence(ctx, m, to_dev(w.frames), w.T, p)
    theta = to_dev(_theta(8, 1).astype(np.float32))
    om = to_dev(learned.sketch_omega(16, 1))
    dmc.learned_start(ctx, 16, 8, om, theta)  # registered for k = 8, used with k = 10
    try:
        with pytest.raises(dmc.DmcError):
            dmc.compress_sequence(ctx, m, to_dev(w.frames), w.T, p)
    finally:
        dmc.learned_start(ctx, 0, 0, None, None)
