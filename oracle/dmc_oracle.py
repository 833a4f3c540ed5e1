"""Plain, slow, float64 CPU oracle of the spatio-temporal mesh compressor
(Arvanitis, Lalos, Moustakas, "Fast Spatio-temporal Compression of Dynamic 3D
Meshes", arXiv 2111.10105).

TEST INFRASTRUCTURE ONLY.  Nothing in the library imports, links or runs this
file; only the tests, the package's smoke check and the benchmark's CPU-baseline
leg do.  It shares no code with the HIP library: it is NumPy/SciPy written from
the paper's equations, one step per function, with no blocking or fusion.

Notation follows the paper (Sec. II-III):  n vertices, a window of T frames
(the paper's k_f), A_c the T x n matrix of coordinate c in {x, y, z}, L the mesh
Laplacian, R_c = A_c A_c^T, U_k the first k eigen-trajectories, delta_c = L A_c^T,
Y_c = U_k^T delta_c^T the projected coefficients, N the anchor index set.

Readings where the paper is silent or ambiguous (each is listed with its reason
in the design notes of the repository):
  * Laplacian default is the normalised form of Eq. (3), I - D^-1 C; Eq. (1),
    D - C, is selectable.
  * The autocorrelation of Eq. (7) is not centred.
  * Q(.) of Eq. (10) is a uniform quantiser per row over [min, max] of the row,
    with the range stored as float32 and the arithmetic done in float64 as
    separate IEEE operations (see `quantise_uniform`).
  * The dictionary and anchors use 16-bit uniform codes (Table I discussion:
    16 bits for anchors and dictionary entries); the dictionary range is [-1, 1].
  * The encoder projects with the dequantised dictionary (the one the decoder
    sees).
  * Eigenvectors are ordered by eigenvalue, largest first (Eq. (5) SVD
    convention); the sign of each is fixed so that its entry of largest
    magnitude is positive (lowest index on an exact tie).
  * A short last window (F not a multiple of T) keeps k_w = min(k, T_w) rows and
    starts from the exact eigenvectors of its own covariance.
  * The anchored system of Eq. (12) is solved in the least-squares sense with
    anchor weight 1, for all T columns at once (the "parallel" variant).

Parity status per function: every public function below is pinned by a test in
tests/test_oracle_*.py against a closed form, an invariant, a library routine,
brute force, or numbers printed in the paper, except `rate_distortion`-style
quality numbers, which the paper reports only on datasets not available here
(parity unpinned for absolute quality).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.csgraph as csgraph
import scipy.sparse.linalg as spla

LAP_UNIFORM = "uniform"            # Eq. (3): delta_i = v_i - mean of first-ring neighbours
LAP_COMBINATORIAL = "combinatorial"  # Eq. (1): L = D - C


# ---------------------------------------------------------------------------
# Sec. II: mesh graph, adjacency (Eq. 2), degrees, Laplacian (Eq. 1, Eq. 3-4)
# ---------------------------------------------------------------------------

def adjacency(n: int, tris: np.ndarray) -> sp.csr_matrix:
    """Binary adjacency C of Eq. (2): C_ij = 1 iff j is in the first ring of i.

    The first ring of i is every vertex sharing a triangle edge with i.  Edges
    seen twice (from two triangles) are merged; self loops are dropped.
    """
    tris = np.asarray(tris, dtype=np.int64)
    if tris.size and (tris.min() < 0 or tris.max() >= n):
        raise ValueError("triangle index out of range")
    a = np.concatenate([tris[:, 0], tris[:, 1], tris[:, 2]])
    b = np.concatenate([tris[:, 1], tris[:, 2], tris[:, 0]])
    keep = a != b
    a, b = a[keep], b[keep]
    rows = np.concatenate([a, b])
    cols = np.concatenate([b, a])
    C = sp.coo_matrix((np.ones(rows.size), (rows, cols)), shape=(n, n)).tocsr()
    C.data[:] = 1.0  # duplicates summed above; binary per Eq. (2)
    C.eliminate_zeros()
    C.sort_indices()
    return C


def degrees(C: sp.csr_matrix) -> np.ndarray:
    """d_i = sum_j C_ij (diagonal of D, Sec. II)."""
    return np.asarray(C.sum(axis=1)).ravel()


def laplacian(n: int, tris: np.ndarray, kind: str = LAP_UNIFORM) -> sp.csr_matrix:
    """Mesh Laplacian.

    uniform       : L = I - D^-1 C, so (L V)_i is Eq. (3)'s delta_i.
    combinatorial : L = D - C (Eq. 1).
    A vertex with no neighbour makes Eq. (3) undefined and is rejected.
    """
    C = adjacency(n, tris)
    d = degrees(C)
    if np.any(d == 0):
        raise ValueError("isolated vertex: Eq. (3) needs at least one neighbour")
    if kind == LAP_UNIFORM:
        return (sp.identity(n, format="csr") - sp.diags(1.0 / d) @ C).tocsr()
    if kind == LAP_COMBINATORIAL:
        return (sp.diags(d) - C).tocsr()
    raise ValueError(f"unknown Laplacian kind {kind!r}")


def delta_coordinates(L: sp.csr_matrix, frames: np.ndarray) -> np.ndarray:
    """Delta coordinates of every frame, delta = L V (Eq. 4), i.e. Eq. (8) per
    coordinate.  frames [T][n][3] -> [T][n][3]."""
    frames = np.asarray(frames, dtype=np.float64)
    return np.stack([L @ frames[t] for t in range(frames.shape[0])], axis=0)


# ---------------------------------------------------------------------------
# Sec. III-A: windows ("blocks" of k_f consecutive frames)
# ---------------------------------------------------------------------------

def windows(F: int, T: int) -> list[tuple[int, int]]:
    """Frame ranges [start, stop) of consecutive windows of T frames; the last
    one is shorter when T does not divide F."""
    if F <= 0 or T <= 0:
        raise ValueError("F and T must be positive")
    return [(s, min(s + T, F)) for s in range(0, F, T)]


def coordinate_matrix(frames_w: np.ndarray, c: int) -> np.ndarray:
    """A_c of Sec. III: T x n matrix holding coordinate c of every vertex of
    every frame of the window."""
    return np.asarray(frames_w[:, :, c], dtype=np.float64)


def autocorrelation(A_c: np.ndarray) -> np.ndarray:
    """R_c = A_c A_c^T (Eq. 7), not centred."""
    return A_c @ A_c.T


# ---------------------------------------------------------------------------
# Eq. (5): symmetric eigendecomposition by cyclic Jacobi, sorted, sign-fixed
# ---------------------------------------------------------------------------

def sign_fix(V: np.ndarray) -> np.ndarray:
    """Make the entry of largest magnitude of every column positive (lowest row
    index on an exact tie)."""
    V = np.array(V, dtype=np.float64, copy=True)
    for j in range(V.shape[1]):
        i = int(np.argmax(np.abs(V[:, j])))  # argmax returns the first maximum
        if V[i, j] < 0:
            V[:, j] = -V[:, j]
    return V


def jacobi_eigh(S: np.ndarray, max_sweeps: int = 100):
    """Eigenpairs of a symmetric matrix by the cyclic Jacobi method.

    Each sweep visits every pair (p, q), p < q, in row order and zeroes S_pq
    with a plane rotation (tangent t = sgn(th) / (|th| + sqrt(th^2 + 1)),
    th = (S_qq - S_pp) / (2 S_pq)).  A pair is skipped once |S_pq| is below
    eps * sqrt(|S_pp S_qq|); the iteration ends after a sweep with no rotation.
    Returns eigenvalues in decreasing order and the matching sign-fixed
    eigenvectors as columns.
    """
    A = np.array(S, dtype=np.float64, copy=True)
    m = A.shape[0]
    if A.shape != (m, m):
        raise ValueError("square matrix expected")
    if not np.allclose(A, A.T, rtol=0, atol=1e-12 * max(1.0, np.abs(A).max())):
        raise ValueError("symmetric matrix expected")
    A = 0.5 * (A + A.T)
    V = np.eye(m)
    eps = np.finfo(np.float64).eps
    tiny = np.finfo(np.float64).tiny
    for _ in range(max_sweeps):
        rotated = False
        for p in range(m - 1):
            for q in range(p + 1, m):
                apq = A[p, q]
                if abs(apq) <= max(eps * math.sqrt(abs(A[p, p] * A[q, q])), tiny):
                    continue
                rotated = True
                th = (A[q, q] - A[p, p]) / (2.0 * apq)
                t = math.copysign(1.0, th) / (abs(th) + math.sqrt(th * th + 1.0))
                c = 1.0 / math.sqrt(t * t + 1.0)
                s = t * c
                # A <- J^T A J with J the rotation in the (p, q) plane
                ap = A[:, p].copy()
                aq = A[:, q].copy()
                A[:, p] = c * ap - s * aq
                A[:, q] = s * ap + c * aq
                rp = A[p, :].copy()
                rq = A[q, :].copy()
                A[p, :] = c * rp - s * rq
                A[q, :] = s * rp + c * rq
                A[p, q] = A[q, p] = 0.0
                vp = V[:, p].copy()
                vq = V[:, q].copy()
                V[:, p] = c * vp - s * vq
                V[:, q] = s * vp + c * vq
        if not rotated:
            break
    lam = np.diag(A).copy()
    order = np.argsort(-lam, kind="stable")
    return lam[order], sign_fix(V[:, order])


# ---------------------------------------------------------------------------
# Sec. II-B, Algorithm 1: orthogonal iterations and the Ritz step
# ---------------------------------------------------------------------------

def orthonormalise(Y: np.ndarray) -> np.ndarray:
    """Thin QR, Q factor with positive diagonal of R (Householder, LAPACK)."""
    Q, Rf = np.linalg.qr(Y)
    s = np.sign(np.diag(Rf))
    s[s == 0] = 1.0
    return Q * s


def oi_residual(R: np.ndarray, Q: np.ndarray) -> float:
    """|| R Q - Q (Q^T R Q) ||_F / ||R||_F: how far span(Q) is from an
    invariant subspace of R."""
    RQ = R @ Q
    nr = np.linalg.norm(R)
    if nr == 0.0:
        return 0.0
    return float(np.linalg.norm(RQ - Q @ (Q.T @ RQ)) / nr)


def orthogonal_iterations(R: np.ndarray, Q0: np.ndarray, tol: float, max_sweeps: int):
    """The inner loop of Algorithm 1: U^(t) = QR(R U^(t-1)).

    Q0 is the start block (the previous window's subspace, or any full-rank
    T x k block).  Every sweep multiplies by R and re-orthonormalises; the loop
    stops after the first sweep whose result has oi_residual <= tol, or after
    max_sweeps.  Returns (Q, sweeps, residual).
    """
    Q = orthonormalise(np.asarray(Q0, dtype=np.float64))
    resid = oi_residual(R, Q)
    sweeps = 0
    for s in range(max_sweeps):
        Q = orthonormalise(R @ Q)
        sweeps = s + 1
        resid = oi_residual(R, Q)
        if resid <= tol:
            break
    return Q, sweeps, resid


def ritz(R: np.ndarray, Q: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Rayleigh-Ritz on span(Q): H = Q^T R Q, H = V diag(mu) V^T (Jacobi),
    U = Q V, columns ordered by mu decreasing, signs fixed as in `sign_fix`."""
    H = Q.T @ R @ Q
    H = 0.5 * (H + H.T)
    mu, V = jacobi_eigh(H)
    return mu, sign_fix(Q @ V)


def exact_subspace(R: np.ndarray, k: int) -> tuple[np.ndarray, np.ndarray]:
    """First k eigenpairs of R by Eq. (5) (Algorithm 1, first block)."""
    lam, U = jacobi_eigh(R)
    return lam[:k], U[:, :k]


# ---------------------------------------------------------------------------
# Eq. (10): uniform quantiser Q(.) and its inverse
# ---------------------------------------------------------------------------

def f32_down(x: float) -> np.float32:
    """Largest float32 <= x."""
    f = np.float32(x)
    if float(f) > x:
        f = np.nextafter(f, np.float32(-np.inf))
    return np.float32(f)


def f32_up(x: float) -> np.float32:
    """Smallest float32 >= x."""
    f = np.float32(x)
    if float(f) < x:
        f = np.nextafter(f, np.float32(np.inf))
    return np.float32(f)


def stored_range(values: np.ndarray) -> tuple[np.float32, np.float32]:
    """(lo, hi) of a set of values, stored as float32 so that lo <= min and
    hi >= max (exact when the values are float32 already)."""
    v = np.asarray(values)
    return f32_down(float(v.min())), f32_up(float(v.max()))


def quantise_uniform(y: np.ndarray, lo: float, hi: float, bits: int) -> np.ndarray:
    """Codes of Q(.) with 2^bits levels over [lo, hi].

    Float64, one IEEE operation at a time:
      s = (2^b - 1) / (hi - lo);  t = (y - lo) * s;
      code = min(2^b - 1, max(0, floor(t + 0.5)))  (round half up).
    A degenerate range (hi == lo) gives code 0 everywhere.
    """
    if not 1 <= bits <= 16:
        raise ValueError("bits must be in 1..16")
    levels = float((1 << bits) - 1)
    lo = np.float64(lo)
    hi = np.float64(hi)
    y = np.asarray(y, dtype=np.float64)
    if hi == lo:
        return np.zeros(y.shape, dtype=np.uint16)
    s = np.float64(levels) / (hi - lo)
    t = (y - lo) * s
    code = np.floor(t + 0.5)
    code = np.minimum(levels, np.maximum(0.0, code))
    return code.astype(np.uint16)


def dequantise_uniform(codes: np.ndarray, lo: float, hi: float, bits: int) -> np.ndarray:
    """Reconstruction points: lo + code * ((hi - lo) / (2^b - 1)), float64."""
    levels = float((1 << bits) - 1)
    lo = np.float64(lo)
    hi = np.float64(hi)
    step = (hi - lo) / np.float64(levels)
    return lo + np.asarray(codes, dtype=np.float64) * step


def quantise_dictionary(U: np.ndarray, bits: int):
    """Dictionary entries (unit eigenvectors, so within [-1, 1]) quantised with
    `bits` over the fixed range [-1, 1]; returns (codes, dequantised).
    bits == 0 keeps the float values."""
    if bits == 0:
        return None, np.asarray(U, dtype=np.float64)
    codes = quantise_uniform(U, -1.0, 1.0, bits)
    return codes, dequantise_uniform(codes, -1.0, 1.0, bits)


# ---------------------------------------------------------------------------
# Encoder (Eq. 8-10, Eq. 12 anchors) for one window
# ---------------------------------------------------------------------------

def project(U_tilde: np.ndarray, delta_c: np.ndarray) -> np.ndarray:
    """Y_c = U^T delta_c^T (Eq. 9) with only the k kept eigen-trajectories:
    U_tilde T x k, delta_c n x T -> k x n."""
    return U_tilde.T @ delta_c.T


def quantise_rows(Y: np.ndarray, bits: int, fp32_data: bool):
    """Eq. (10) on the kept rows: per row r, range [lo_r, hi_r] over the row,
    codes by `quantise_uniform`.  Returns (codes [k][n] uint16, ranges [k][2]
    float32, dequantised [k][n] float64).  bits == 0 keeps the float values."""
    k = Y.shape[0]
    if bits == 0:
        return None, None, np.asarray(Y, dtype=np.float64)
    codes = np.empty(Y.shape, dtype=np.uint16)
    ranges = np.empty((k, 2), dtype=np.float32)
    deq = np.empty(Y.shape, dtype=np.float64)
    for r in range(k):
        row = Y[r].astype(np.float32) if fp32_data else Y[r]
        lo, hi = stored_range(row)
        ranges[r] = (lo, hi)
        codes[r] = quantise_uniform(row, lo, hi, bits)
        deq[r] = dequantise_uniform(codes[r], lo, hi, bits)
    return codes, ranges, deq


def anchor_values(frames_w: np.ndarray, anchors: np.ndarray, c: int) -> np.ndarray:
    """I_nc A_c^T of Eq. (12): the anchor rows of coordinate c, n_c x T."""
    return np.asarray(frames_w[:, anchors, c], dtype=np.float64).T


def encode_window(L, frames_w, anchors, k, bits, *, dict_bits=16, anchor_bits=16,
                  q_start=None, omega=None, learned=None, oi_tol=1e-12, oi_max_sweeps=200,
                  fp32_data=False):
    """One window of the encoder.

    q_start None -> exact eigenvectors of each R_c (Algorithm 1, first block);
    otherwise a [3][T][k] start block for orthogonal iterations followed by the
    Ritz step.  omega ([T][k]) instead starts every coordinate from the sketch
    R_c omega; learned = (Omega [T][32], theta) from the row-wise perceptron's
    prediction on the sketch (oracle.mlp_oracle.predict_start).  Returns a dict with the dictionary, coefficients, codes,
    anchor codes and per-coordinate iteration counts.
    """
    frames_w = np.asarray(frames_w)
    T = frames_w.shape[0]
    kw = min(k, T)
    delta = delta_coordinates(L, frames_w)
    rec = {"T": T, "k": kw, "bits": bits, "dict_bits": dict_bits,
           "anchor_bits": anchor_bits, "U": [], "U_tilde": [], "U_codes": [],
           "Y": [], "codes": [], "ranges": [], "Y_hat": [], "anchor_codes": [],
           "anchor_range": [], "A_hat": [], "sweeps": [], "resid": [], "eig": []}
    for c in range(3):
        A_c = coordinate_matrix(frames_w, c)
        R = autocorrelation(A_c)
        if learned is not None:
            from .mlp_oracle import predict_start
            Q0 = predict_start(R, learned[0], learned[1], kw)
            Q, sweeps, resid = orthogonal_iterations(R, Q0, oi_tol, oi_max_sweeps)
            lam, U = ritz(R, Q)
        elif omega is not None:
            Q, sweeps, resid = orthogonal_iterations(R, R @ omega[:, :kw], oi_tol, oi_max_sweeps)
            lam, U = ritz(R, Q)
        elif q_start is None:
            lam, U = exact_subspace(R, kw)
            sweeps, resid = 0, oi_residual(R, U)
        else:
            Q, sweeps, resid = orthogonal_iterations(R, q_start[c][:, :kw], oi_tol,
                                                     oi_max_sweeps)
            lam, U = ritz(R, Q)
        ucodes, Ut = quantise_dictionary(U, dict_bits)
        Y = project(Ut, delta[:, :, c].T)
        codes, ranges, Yh = quantise_rows(Y, bits, fp32_data)
        a = anchor_values(frames_w, anchors, c)
        if anchor_bits == 0:
            acodes, arange, ah = None, None, a
        else:
            lo, hi = stored_range(a.astype(np.float32) if fp32_data else a)
            acodes = quantise_uniform(a, lo, hi, anchor_bits)
            arange = np.array([lo, hi], dtype=np.float32)
            ah = dequantise_uniform(acodes, lo, hi, anchor_bits)
        for key, val in (("U", U), ("U_tilde", Ut), ("U_codes", ucodes), ("Y", Y),
                         ("codes", codes), ("ranges", ranges), ("Y_hat", Yh),
                         ("anchor_codes", acodes), ("anchor_range", arange),
                         ("A_hat", ah), ("sweeps", sweeps), ("resid", resid),
                         ("eig", lam)):
            rec[key].append(val)
    return rec


# ---------------------------------------------------------------------------
# Decoder (Eq. 12): anchored least squares, all frames of a window at once
# ---------------------------------------------------------------------------

def selection(n: int, anchors: np.ndarray) -> sp.csr_matrix:
    """I_nc of Eq. (12): the rows of the n x n identity indexed by N."""
    anchors = np.asarray(anchors, dtype=np.int64)
    m = anchors.size
    return sp.csr_matrix((np.ones(m), (np.arange(m), anchors)), shape=(m, n))


def normal_matrix(L: sp.csr_matrix, anchors: np.ndarray) -> sp.csc_matrix:
    """L^T L + I_nc^T I_nc: the normal equations of the stacked system (12)."""
    P = selection(L.shape[0], anchors)
    return (L.T @ L + P.T @ P).tocsc()


class AnchoredSolver:
    """Least-squares solution of [L; I_nc] X = [B; A_N] (Eq. 12) through the
    normal equations, factorised once per mesh by sparse LU (SuperLU)."""

    def __init__(self, L: sp.csr_matrix, anchors: np.ndarray):
        self.L = L
        self.anchors = np.asarray(anchors, dtype=np.int64)
        self.P = selection(L.shape[0], self.anchors)
        M = normal_matrix(L, self.anchors)
        # L^T L annihilates every vector constant on a connected component, so
        # the normal matrix is singular unless each component holds an anchor
        self._check_nonsingular()
        self.lu = spla.splu(M)

    def _check_nonsingular(self):
        C = abs(self.L) > 0
        ncomp, labels = csgraph.connected_components(C, directed=False)
        anchored = np.zeros(ncomp, dtype=bool)
        anchored[labels[self.anchors]] = True
        if not anchored.all():
            raise np.linalg.LinAlgError("a connected component has no anchor: "
                                        "the system of Eq. (12) is singular")

    def solve(self, B: np.ndarray, A_N: np.ndarray) -> np.ndarray:
        """B: n x m right-hand side of the L rows; A_N: n_c x m anchor values."""
        rhs = self.L.T @ B + self.P.T @ A_N
        return self.lu.solve(np.asarray(rhs, dtype=np.float64))


def back_project(U_tilde: np.ndarray, Y_hat: np.ndarray) -> np.ndarray:
    """delta-tilde_c = (U Y-hat)^T (Eq. 11/12 right-hand side), n x T."""
    return (U_tilde @ Y_hat).T


def decode_window(solver: AnchoredSolver, rec) -> np.ndarray:
    """Reconstruct the window's frames [T][n][3] from one encoded record."""
    T = rec["T"]
    out = np.empty((T, solver.L.shape[0], 3))
    for c in range(3):
        B = back_project(rec["U_tilde"][c], rec["Y_hat"][c])
        out[:, :, c] = solver.solve(B, rec["A_hat"][c]).T
    return out


# ---------------------------------------------------------------------------
# Whole sequence (Sec. III-A) and reporting (Eq. 13, error)
# ---------------------------------------------------------------------------

def compress_sequence(n, tris, frames, anchors, T, k, bits, *, laplacian_kind=LAP_UNIFORM,
                      dict_bits=16, anchor_bits=16, first_start=None, init="prev",
                      starts=None, omega=None, learned=None, oi_tol=1e-12, oi_max_sweeps=200,
                      decode=True, fp32_data=False):
    """Encode (and decode) every window.  Start of each full window's
    orthogonal iterations, by `init`:
      "prev"   window w > 0 from window w-1's U_k (Algorithm 1); window 0 from
               `first_start` ([3][T][k]) or, if None, its exact eigenvectors;
      "random" window w from starts[w] ([nw][3][T][k]);
      "sketch" every window from R_c omega (omega [T][k]);
      "exact"  every window from its exact eigenvectors (Eq. 5);
      "learned" every window from the perceptron's prediction, learned =
               (Omega [T][32], theta).
    A short last window starts from its own exact eigenvectors.
    Returns (records, reconstruction or None)."""
    L = laplacian(n, tris, laplacian_kind)
    frames = np.asarray(frames)
    recs = []
    prev = first_start
    for wi, (s, e) in enumerate(windows(frames.shape[0], T)):
        fw = frames[s:e]
        full = (e - s) == T
        start, om = None, None
        if full and init == "prev":
            start = prev
        elif full and init == "random":
            start = starts[wi]
        elif full and init == "sketch":
            om = omega
        lrn = learned if (full and init == "learned") else None
        rec = encode_window(L, fw, anchors, k, bits, dict_bits=dict_bits,
                            anchor_bits=anchor_bits, q_start=start, omega=om, learned=lrn,
                            oi_tol=oi_tol,
                            oi_max_sweeps=oi_max_sweeps, fp32_data=fp32_data)
        rec["start"] = s
        recs.append(rec)
        prev = np.stack(rec["U"], axis=0)
    if not decode:
        return recs, None
    solver = AnchoredSolver(L, anchors)
    out = np.empty(frames.shape, dtype=np.float64)
    for rec in recs:
        s = rec["start"]
        out[s:s + rec["T"]] = decode_window(solver, rec)
    return recs, out


def nmse(X: np.ndarray, Y: np.ndarray) -> float:
    """sum (X - Y)^2 / sum Y^2 over every vertex, frame and coordinate."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    return float(np.sum((X - Y) ** 2) / np.sum(Y ** 2))


def bpvf(n: int, F: int, n_anchors: int, window_shapes, bits: int,
         anchor_bits: int = 16, dict_bits: int = 16, raw_bits: int = 64) -> dict:
    """Bits per vertex per frame for one coordinate (Eq. 13 and its
    discussion), for what this encoder actually sends:
      q   : coefficient codes, bits * k_w * n per window
      q_r : their row ranges, 2 float32 per kept row per window
      q_a : anchor codes, anchor_bits * n_c per frame (+ 2 float32 per window)
      q_d : dictionary, dict_bits * T_w * k_w per window
      q_s : the sum.
    A part whose bit count is 0 is sent as raw values of raw_bits each and
    has no range.  window_shapes: iterable of (T_w, k_w)."""
    vf = float(n * F)
    shapes = list(window_shapes)
    q = sum((bits or raw_bits) * kw * n for (_tw, kw) in shapes) / vf
    q_r = sum(64 * kw for (_tw, kw) in shapes) / vf if bits else 0.0
    q_a = ((anchor_bits or raw_bits) * n_anchors * F + (64 * len(shapes) if anchor_bits else 0)) / vf
    q_d = sum((dict_bits or raw_bits) * tw * kw for (tw, kw) in shapes) / vf
    return {"q": q, "q_r": q_r, "q_a": q_a, "q_d": q_d, "q_s": q + q_r + q_a + q_d}


def bpvf_paper(n: int, k: int, n_anchors: int, n_b: int, k_f: int,
               bits_anchor: int = 16, bits_dict: int = 16) -> dict:
    """The side-information terms of Eq. (13) as printed: q_a = b n_c k / (n k),
    q_d = b n_b^2 k_f^2 / (n k), with k the number of frames."""
    return {"q_a": bits_anchor * n_anchors * k / (n * k),
            "q_d": bits_dict * n_b * n_b * k_f * k_f / (n * k)}
