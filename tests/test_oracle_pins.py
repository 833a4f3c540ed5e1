"""Pins of the float64 CPU oracle against facts the paper and the mathematics
fix (closed forms, invariants, textbook routines, brute force, and the
numbers printed in Table I).  CPU only."""
import itertools
import json
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
from synth import animate, meshes

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- Laplacian

def _brute_delta(n, tris, V, kind):
    """Eq. (3) / Eq. (1) written with explicit neighbour sets built from the
    triangle list (no sparse algebra)."""
    ring = [set() for _ in range(n)]
    for a, b, c in tris:
        for x, y in ((a, b), (b, c), (c, a)):
            if x != y:
                ring[x].add(y)
                ring[y].add(x)
    out = np.empty_like(V)
    for i in range(n):
        nb = sorted(ring[i])
        s = sum(V[j] for j in nb)
        if kind == O.LAP_UNIFORM:
            out[i] = V[i] - s / len(nb)
        else:
            out[i] = len(nb) * V[i] - s
    return out


@pytest.mark.parametrize("kind", [O.LAP_UNIFORM, O.LAP_COMBINATORIAL])
@pytest.mark.parametrize("mesh", ["ico1", "grid", "torus"])
def test_laplacian_matches_neighbour_sets(kind, mesh):
    v, t = {"ico1": meshes.icosphere(1), "grid": meshes.grid(5, 4),
            "torus": meshes.torus(6, 5)}[mesh]
    L = O.laplacian(v.shape[0], t, kind)
    rng = np.random.default_rng(0)
    V = rng.standard_normal((v.shape[0], 3))
    np.testing.assert_allclose(L @ V, _brute_delta(v.shape[0], t, V, kind), atol=1e-13)


def test_laplacian_rows_sum_to_zero_and_translation():
    v, t = meshes.icosphere(2)
    n = v.shape[0]
    Lu = O.laplacian(n, t, O.LAP_UNIFORM)
    Lc = O.laplacian(n, t, O.LAP_COMBINATORIAL)
    assert np.max(np.abs(Lc @ np.ones(n))) == 0.0
    assert np.max(np.abs(Lu @ np.ones(n))) <= 4 * np.finfo(float).eps
    # symmetric combinatorial form; D L_unif = L_comb
    assert abs(Lc - Lc.T).max() == 0.0
    d = O.degrees(O.adjacency(n, t))
    assert abs(sp.diags(d) @ Lu - Lc).max() < 1e-14
    # translating every frame leaves the delta coordinates unchanged
    fr = animate.bend_twist(v, 4, seed=3)
    shift = np.array([0.3, -1.25, 2.0])
    d0 = O.delta_coordinates(Lu, fr)
    d1 = O.delta_coordinates(Lu, fr + shift)
    assert np.max(np.abs(d0 - d1)) < 1e-13


def test_isolated_vertex_rejected():
    v, t = meshes.icosphere(0)
    with pytest.raises(ValueError):
        O.laplacian(v.shape[0] + 1, t)


def test_adjacency_degrees_closed_surface():
    # icosphere: 12 degree-5 vertices, all others degree 6; 2E = sum of degrees
    v, t = meshes.icosphere(2)
    d = O.degrees(O.adjacency(v.shape[0], t))
    assert np.sum(d == 5) == 12 and np.all((d == 5) | (d == 6))
    assert d.sum() == 3 * t.shape[0]  # closed manifold: E = 3F/2


# ---------------------------------------------------------------- eigen (Eq. 5)

@pytest.mark.parametrize("m,seed", [(5, 0), (16, 1), (32, 2)])
def test_jacobi_matches_lapack(m, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, 3 * m))
    S = A @ A.T
    lam, V = O.jacobi_eigh(S)
    ref = np.linalg.eigh(S)[0][::-1]
    assert np.max(np.abs(lam - ref)) <= 1e-12 * ref[0]
    assert np.max(np.abs(V.T @ V - np.eye(m))) < 1e-13
    assert np.max(np.abs(S @ V - V * lam)) <= 1e-12 * ref[0]
    assert np.all(np.diff(lam) <= 0)


def test_sign_rule():
    V = np.array([[0.1, -0.5], [-0.9, 0.5], [0.2, 0.1]])
    W = O.sign_fix(V)
    assert W[1, 0] > 0          # largest magnitude entry made positive
    assert W[0, 1] > 0          # tie between rows 0 and 1: lowest row wins


def test_trace_equals_eigen_sum_and_frobenius():
    v, t = meshes.icosphere(2)
    fr = animate.bend_twist(v, 12, seed=5)
    for c in range(3):
        A = O.coordinate_matrix(fr, c)
        R = O.autocorrelation(A)
        lam, _ = O.jacobi_eigh(R)
        assert abs(lam.sum() - np.sum(A * A)) <= 1e-12 * np.sum(A * A)


def test_static_mesh_closed_form():
    """All frames equal: R = |a|^2 11^T, u_1 = 1/sqrt(T), Y_1 = sqrt(T) (L a)^T,
    and k = 1 with raw values reconstructs exactly."""
    v, t = meshes.icosphere(2)
    n, T = v.shape[0], 8
    fr = np.broadcast_to(v, (T, n, 3)).copy()
    L = O.laplacian(n, t)
    anchors = animate.choose_anchors(n, 3, seed=1)
    rec = O.encode_window(L, fr, anchors, 1, 0, dict_bits=0, anchor_bits=0)
    for c in range(3):
        a = v[:, c]
        assert abs(rec["eig"][c][0] - T * a @ a) <= 1e-12 * T * a @ a
        np.testing.assert_allclose(rec["U"][c][:, 0], np.full(T, 1 / np.sqrt(T)), atol=1e-14)
        np.testing.assert_allclose(rec["Y"][c][0], np.sqrt(T) * (L @ a), atol=1e-13)
    out = O.decode_window(O.AnchoredSolver(L, anchors), rec)
    assert np.max(np.abs(out - fr)) < 1e-10


def test_linear_motion_rank_two():
    """A(t) = a + t v: rank R <= 2, k = 2 (raw) reconstructs to round-off."""
    v, t = meshes.icosphere(2)
    n, T = v.shape[0], 10
    vel = np.random.default_rng(2).standard_normal((n, 3)) * 0.05
    fr = np.stack([v + s * vel for s in range(T)])
    L = O.laplacian(n, t)
    anchors = animate.choose_anchors(n, 4, seed=3)
    rec = O.encode_window(L, fr, anchors, 2, 0, dict_bits=0, anchor_bits=0)
    for c in range(3):
        lam = rec["eig"][c]
        assert lam[1] > 0
    full = O.encode_window(L, fr, anchors, T, 0, dict_bits=0, anchor_bits=0)
    for c in range(3):
        assert full["eig"][c][2] <= 1e-12 * full["eig"][c][0]
    out = O.decode_window(O.AnchoredSolver(L, anchors), rec)
    assert np.max(np.abs(out - fr)) < 1e-9


# ---------------------------------------------------------------- Algorithm 1

def _sin_angle(U, Q):
    """Largest principal angle (sine) between span(U) and span(Q), both
    orthonormal: || (I - U U^T) Q ||_2."""
    return np.linalg.norm(Q - U @ (U.T @ Q), 2)


@pytest.mark.parametrize("level,T,k", [(1, 8, 2), (2, 16, 1), (3, 32, 4)])
def test_oi_subspace_matches_jacobi(level, T, k):
    v, t = meshes.icosphere(level)
    fr = animate.bend_twist(v, T, seed=10 + level, noise_var=1e-6)
    for c in range(3):
        R = O.autocorrelation(O.coordinate_matrix(fr, c))
        lam, U = O.jacobi_eigh(R)
        gap = lam[k - 1] / lam[k]
        assert gap >= 10, gap  # test is only meaningful with a gap
        Q0 = animate.gaussian_subspace(T, k, seed=7)[c]
        Q, sweeps, resid = O.orthogonal_iterations(R, Q0, 1e-13, 500)
        assert resid <= 1e-13
        assert np.max(np.abs(Q.T @ Q - np.eye(k))) < 1e-14
        assert _sin_angle(U[:, :k], Q) < 1e-10
        mu, Uk = O.ritz(R, Q)
        np.testing.assert_allclose(mu, lam[:k], rtol=1e-10)
        # canonical (sorted, sign-fixed) Ritz vectors equal the eigenvectors
        assert np.max(np.abs(Uk - U[:, :k])) < 1e-8


def test_oi_warm_start_identical_windows_one_sweep():
    v, t = meshes.icosphere(2)
    fr = animate.bend_twist(v, 16, seed=4, noise_var=1e-6)
    R = O.autocorrelation(O.coordinate_matrix(fr, 0))
    Q0 = animate.gaussian_subspace(16, 4, seed=1)[0]
    Q, s1, _ = O.orthogonal_iterations(R, Q0, 1e-12, 500)
    _, Uk = O.ritz(R, Q)
    _, s2, r2 = O.orthogonal_iterations(R, Uk, 1e-12, 500)
    assert s1 > 1 and s2 == 1 and r2 <= 1e-12


def test_oi_residual_measures_invariance():
    rng = np.random.default_rng(3)
    A = rng.standard_normal((6, 30))
    R = A @ A.T
    lam, U = O.jacobi_eigh(R)
    assert O.oi_residual(R, U[:, :3]) < 1e-14
    Q = O.orthonormalise(rng.standard_normal((6, 3)))
    assert O.oi_residual(R, Q) > 1e-3


# ---------------------------------------------------------------- quantiser (Eq. 10)

def _exact_code(y, lo, hi, bits):
    """floor((y - lo) (2^b - 1) / (hi - lo) + 1/2) in exact rational arithmetic,
    clamped."""
    lv = (1 << bits) - 1
    t = (Fraction(float(y)) - Fraction(float(lo))) * lv / (Fraction(float(hi)) - Fraction(float(lo)))
    c = (t + Fraction(1, 2)).__floor__()
    return min(lv, max(0, c))


@pytest.mark.parametrize("bits", [1, 4, 10, 12, 16])
def test_quantiser_against_exact_rationals(bits):
    rng = np.random.default_rng(bits)
    y = rng.standard_normal(2000).astype(np.float32)
    lo, hi = O.stored_range(y)
    codes = O.quantise_uniform(y, lo, hi, bits)
    exact = np.array([_exact_code(v, lo, hi, bits) for v in y])
    # the float64 operation sequence may differ from exact rounding only on a
    # value within a few ulps of a half-step boundary
    diff = codes.astype(np.int64) - exact
    assert np.all(np.abs(diff) <= 1)
    assert np.mean(diff != 0) < 1e-3
    assert codes.min() == 0 and codes.max() == (1 << bits) - 1


def test_quantiser_error_bound_and_degenerate():
    rng = np.random.default_rng(1)
    y = rng.uniform(-3, 5, 5000)
    for bits in (2, 8, 12, 16):
        lo, hi = O.stored_range(y)
        yh = O.dequantise_uniform(O.quantise_uniform(y, lo, hi, bits), lo, hi, bits)
        step = (float(hi) - float(lo)) / ((1 << bits) - 1)
        assert np.max(np.abs(yh - y)) <= 0.5 * step * (1 + 1e-9)
    c = O.quantise_uniform(np.full(10, 2.5), 2.5, 2.5, 12)
    assert np.all(c == 0)


def test_quantiser_power_of_two_scaling_invariance():
    rng = np.random.default_rng(9)
    y = rng.standard_normal(4000).astype(np.float32)
    lo, hi = O.stored_range(y)
    c1 = O.quantise_uniform(y, lo, hi, 12)
    y4 = (y * np.float32(4.0)).astype(np.float32)
    lo4, hi4 = O.stored_range(y4)
    c4 = O.quantise_uniform(y4, lo4, hi4, 12)
    assert np.array_equal(c1, c4)


def test_stored_range_brackets_float64_values():
    rng = np.random.default_rng(4)
    y = rng.standard_normal(1000)
    lo, hi = O.stored_range(y)
    assert float(lo) <= y.min() and float(hi) >= y.max()
    assert np.float32(lo) == lo and np.float32(hi) == hi
    assert np.nextafter(lo, np.float32(np.inf)) > y.min()
    assert np.nextafter(hi, np.float32(-np.inf)) < y.max()


# ---------------------------------------------------------------- decoder (Eq. 12)

def test_full_rank_reproduces_input():
    """k = T with raw coefficients, dictionary and anchors reproduces the input
    to round-off (no information is dropped)."""
    v, t = meshes.icosphere(2)
    fr = animate.bend_twist(v, 12, seed=8)
    _, out = O.compress_sequence(v.shape[0], t, fr, animate.choose_anchors(v.shape[0], 3, 1),
                                 12, 12, 0, dict_bits=0, anchor_bits=0)
    assert O.nmse(out, fr) < 1e-20


@pytest.mark.parametrize("kind", [O.LAP_UNIFORM, O.LAP_COMBINATORIAL])
def test_normal_equations_match_dense_lstsq(kind):
    v, t = meshes.torus(8, 7)
    n = v.shape[0]
    L = O.laplacian(n, t, kind)
    anchors = animate.choose_anchors(n, 4, seed=2)
    rng = np.random.default_rng(0)
    B = rng.standard_normal((n, 5))
    A_N = rng.standard_normal((4, 5))
    X = O.AnchoredSolver(L, anchors).solve(B, A_N)
    stacked = np.vstack([L.toarray(), O.selection(n, anchors).toarray()])
    Xd = np.linalg.lstsq(stacked, np.vstack([B, A_N]), rcond=None)[0]
    assert np.max(np.abs(X - Xd)) < 1e-9
    # one column at a time ("serial" variant) gives the same as all at once
    for j in range(5):
        xj = O.AnchoredSolver(L, anchors).solve(B[:, j:j + 1], A_N[:, j:j + 1])
        assert np.max(np.abs(xj[:, 0] - X[:, j])) < 1e-12


def test_unanchored_component_is_singular():
    v, t = meshes.disjoint_union(meshes.icosphere(1), meshes.icosphere(1))
    L = O.laplacian(v.shape[0], t)
    with pytest.raises(np.linalg.LinAlgError):
        O.AnchoredSolver(L, np.array([0, 1], dtype=np.int32))  # both in part one
    O.AnchoredSolver(L, np.array([0, 50], dtype=np.int32))


def test_translation_recovered_through_anchors():
    """Adding c(t) to every vertex leaves the delta part unchanged; the anchors
    carry the translation, and the decode recovers it exactly (raw values)."""
    v, t = meshes.icosphere(2)
    n, T = v.shape[0], 8
    fr = animate.bend_twist(v, T, seed=6)
    shift = np.outer(np.arange(T), [0.5, -0.2, 1.0])[:, None, :]
    anchors = animate.choose_anchors(n, 5, seed=5)
    _, out0 = O.compress_sequence(n, t, fr, anchors, T, T, 0, dict_bits=0, anchor_bits=0)
    _, out1 = O.compress_sequence(n, t, fr + shift, anchors, T, T, 0, dict_bits=0, anchor_bits=0)
    assert np.max(np.abs((out1 - out0) - shift)) < 1e-9


def test_vertex_relabelling_permutes_output():
    v, t = meshes.icosphere(2)
    n, T = v.shape[0], 8
    fr = animate.bend_twist(v, T, seed=12)
    anchors = animate.choose_anchors(n, 5, seed=2)
    perm = np.random.default_rng(3).permutation(n)     # new index -> old index
    inv = np.argsort(perm)                              # old index -> new index
    t2 = inv[t].astype(np.int32)
    _, out = O.compress_sequence(n, t, fr, anchors, T, 4, 12)
    _, out2 = O.compress_sequence(n, t2, fr[:, perm], np.sort(inv[anchors]).astype(np.int32),
                                  T, 4, 12)
    assert np.max(np.abs(out2 - out[:, perm])) < 1e-9


def test_time_reversal():
    v, t = meshes.icosphere(2)
    n, T = v.shape[0], 10
    fr = animate.bend_twist(v, T, seed=13)
    anchors = animate.choose_anchors(n, 5, seed=2)
    _, out = O.compress_sequence(n, t, fr, anchors, T, 5, 0, dict_bits=0, anchor_bits=0)
    _, outr = O.compress_sequence(n, t, fr[::-1], anchors, T, 5, 0, dict_bits=0, anchor_bits=0)
    assert np.max(np.abs(outr[::-1] - out)) < 1e-9


def test_windows_and_ragged_tail():
    assert O.windows(10, 4) == [(0, 4), (4, 8), (8, 10)]
    assert O.windows(8, 8) == [(0, 8)]
    v, t = meshes.torus(10, 8)
    fr = animate.rbf_skinning(v, 21, 3, seed=1, dtype=np.float64)
    anchors = animate.choose_anchors(v.shape[0], 3, seed=1)
    recs, out = O.compress_sequence(v.shape[0], t, fr, anchors, 8, 6, 12)
    assert [r["T"] for r in recs] == [8, 8, 5]
    assert [r["k"] for r in recs] == [6, 6, 5]
    assert O.nmse(out, fr) < 1e-4


def test_blocks_with_one_window_equal_single_window():
    """n_b = 1 is the whole-sequence case (Sec. III-A)."""
    v, t = meshes.icosphere(2)
    n, T = v.shape[0], 12
    fr = animate.bend_twist(v, T, seed=21)
    anchors = animate.choose_anchors(n, 4, seed=2)
    L = O.laplacian(n, t)
    rec = O.encode_window(L, fr, anchors, 6, 12)
    out1 = O.decode_window(O.AnchoredSolver(L, anchors), rec)
    _, out2 = O.compress_sequence(n, t, fr, anchors, T, 6, 12)
    assert np.array_equal(out1, out2)


# ---------------------------------------------------------------- Eq. 13 / Table I

def test_table1_side_information():
    g = json.load(open(os.path.join(GOLDEN, "table1_bpvf.json")))
    hs = g["models"]["Handstand"]
    p = O.bpvf_paper(hs["n"], hs["k"], hs["n_c"], 1, hs["k"])
    assert round(p["q_a"], 4) == hs["pca_qp"]["q_a"]
    assert round(p["q_d"], 4) == hs["pca_qp"]["q_d"]
    sb = g["models"]["Samba"]
    p = O.bpvf_paper(sb["n"], sb["k"], sb["n_c"], 1, sb["k"])
    assert round(p["q_d"], 4) == sb["pca_qp"]["q_d"]
    # Samba's printed q_a (0.1595) fits 1% anchors only to ~1e-3 (printed rounding)
    assert abs(p["q_a"] - sb["pca_qp"]["q_a"]) < 1.5e-3
    # q_s = q + q_a + q_d in every column of the table
    for m in g["models"].values():
        for col in ("pca_qp", "blocks"):
            e = m[col]
            assert abs(e["q"] + e["q_a"] + e["q_d"] - e["q_s"]) <= 1e-3


def test_bpvf_reproduces_table1_side_information():
    """bpvf() on the shape of Table I's PCA+qs/qp column (one window spanning
    all F = T = 175 frames, every frame's eigen-trajectory kept, 1% anchors,
    16-bit anchors and dictionary, Sec. IV) gives the printed q_a and q_d to
    the table's four digits; our range side information (two float32 per
    window and coordinate) is the only extra and stays below the printed
    rounding."""
    g = json.load(open(os.path.join(GOLDEN, "table1_bpvf.json")))
    hs = g["models"]["Handstand"]
    n, F, nc = hs["n"], hs["k"], hs["n_c"]
    b = O.bpvf(n, F, nc, [(F, F)], bits=12)
    assert round(b["q_a"], 4) == hs["pca_qp"]["q_a"]
    assert round(b["q_d"], 4) == hs["pca_qp"]["q_d"]
    assert b["q_a"] - 16 * nc / n == pytest.approx(64 / (n * F))
    sb = g["models"]["Samba"]
    b = O.bpvf(sb["n"], sb["k"], sb["n_c"], [(sb["k"], sb["k"])], bits=12)
    assert round(b["q_d"], 4) == sb["pca_qp"]["q_d"]


def test_bpvf_counts_the_bits_of_each_part():
    """Brute-force count of the bits a small sequence's records carry, summed
    part by part, against bpvf()'s per-vertex-frame figures."""
    n, F, nc = 1000, 20, 10
    shapes = [(8, 4), (8, 4), (4, 4)]
    bits = {"q": 0, "q_r": 0, "q_a": 0, "q_d": 0}
    for tw, kw in shapes:
        for _c in range(1):  # one coordinate
            for _r in range(kw):
                bits["q"] += sum(12 for _ in range(n))
                bits["q_r"] += 2 * 32
            bits["q_a"] += sum(16 for _ in range(tw * nc)) + 2 * 32
            bits["q_d"] += sum(16 for _ in range(tw * kw))
    b = O.bpvf(n, F, nc, shapes, bits=12)
    for key, v in bits.items():
        assert b[key] == pytest.approx(v / (n * F))
    assert b["q_s"] == pytest.approx(sum(bits.values()) / (n * F))
    # raw parts: float32 values, no ranges
    raw = O.bpvf(n, F, nc, shapes, bits=0, anchor_bits=0, dict_bits=0, raw_bits=32)
    assert raw["q"] == pytest.approx(32 * 12 * n / (n * F)) and raw["q_r"] == 0.0
    assert raw["q_a"] == pytest.approx(32 * nc * F / (n * F))


def test_nmse_definition():
    X = np.ones((2, 3, 3))
    Y = np.full((2, 3, 3), 2.0)
    assert O.nmse(X, Y) == pytest.approx(18 / 72)


def test_dictionary_quantiser_range():
    rng = np.random.default_rng(0)
    U = O.orthonormalise(rng.standard_normal((16, 5)))
    codes, Ut = O.quantise_dictionary(U, 16)
    assert codes.dtype == np.uint16
    assert np.max(np.abs(Ut - U)) <= 1.0 / 65535 * (1 + 1e-9)
    # exact integer reference for a few entries
    for (i, j) in itertools.islice(itertools.product(range(16), range(5)), 20):
        assert codes[i, j] == _exact_code(U[i, j], -1.0, 1.0, 16) or \
            abs(int(codes[i, j]) - _exact_code(U[i, j], -1.0, 1.0, 16)) <= 1


@pytest.mark.parametrize("level,F,T,k", [(1, 16, 8, 2), (2, 32, 16, 1), (3, 64, 32, 4)])
def test_sequence_start_modes_reach_the_exact_subspace(level, F, T, k):
    """Every start of the orthogonal iterations (previous window, per-window
    Gaussian block, sketch R_c Omega) converges on gapped windows to the
    window's exact eigenvectors (Jacobi, itself pinned to LAPACK), so the
    records of all modes carry the same dictionary."""
    v, t = meshes.icosphere(level)
    fr = animate.bend_twist(v, F, seed=10 + level, noise_var=1e-6)
    anchors = np.arange(0, v.shape[0], max(1, v.shape[0] // 6))
    nw = F // T
    starts = np.stack([animate.gaussian_subspace(T, k, seed=50 + i) for i in range(nw)])
    omega = animate.gaussian_subspace(T, k, seed=60)[0]
    runs = {}
    for init in ("exact", "prev", "random", "sketch"):
        recs, _ = O.compress_sequence(v.shape[0], t, fr, anchors, T, k, 12, init=init,
                                      first_start=starts[0], starts=starts, omega=omega,
                                      oi_tol=1e-14, decode=False)
        runs[init] = recs
    for w in range(nw):
        for c in range(3):
            U_ex = runs["exact"][w]["U"][c]
            lam, Uj = O.jacobi_eigh(O.autocorrelation(O.coordinate_matrix(fr[w * T:(w + 1) * T], c)))
            assert np.max(np.abs(U_ex - Uj[:, :k] * np.sign(Uj[np.argmax(np.abs(Uj[:, :k]), axis=0),
                                                              range(k)]))) < 1e-12
            for init in ("prev", "random", "sketch"):
                assert runs[init][w]["sweeps"][c] >= 1
                assert _sin_angle(U_ex, runs[init][w]["U"][c]) < 1e-10
                assert np.max(np.abs(runs[init][w]["U"][c] - U_ex)) < 1e-8
    assert all(s == [0, 0, 0] for s in (r["sweeps"] for r in runs["exact"]))
