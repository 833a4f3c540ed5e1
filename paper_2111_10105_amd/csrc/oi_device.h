// Orthogonal iterations (Algorithm 1) with a Rayleigh-Ritz step and the
// dictionary quantiser, for a chain of windows, on one wavefront per
// coordinate (the problem is T <= 64 rows: one lane per row, and a workgroup
// barrier of a single wave costs only the wait for its own LDS traffic).
// Everything lives in LDS in float64:
//   C.Q products on the FP64 matrix cores (v_mfma_f64_16x16x4f64),
//   thin QR by CholeskyQR2 on column-scaled blocks (the columns of R Q differ in
//   norm by the eigenvalue spread, which column scaling removes without
//   changing the Q factor), Gram accumulated in float64, k x k Cholesky,
//   wavefront-shuffle reductions; a pivot breakdown switches that sweep to
//   shifted CholeskyQR3, and a second breakdown (an exactly rank-deficient
//   block) to Gram-Schmidt run twice with completion of the missing
//   directions from the identity;
//   eigenvectors of the k x k Ritz matrix (and of the full T x T matrix for an
//   exact start, Eq. 5) by parallel cyclic Jacobi.
#pragma once
#include <type_traits>

#include "dmc_internal.h"
#include "wave_ops.h"

namespace dmc {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int NT = 64;  // threads per workgroup: one wavefront

// Row strides are padded to an odd number of doubles so that the lanes of a
// wavefront walking down one column hit different LDS banks.
template <int TMAX, int KMAX>
struct OiSmem {
  static constexpr int LR = TMAX + 1;  // stride of R, A, V
  static constexpr int LQ = KMAX + 1;  // stride of Q, Y
  double R[TMAX * LR];
  double A[TMAX * LR];   // Jacobi work matrix; Gram / Cholesky factor; Ritz H
  double V[TMAX * LR];   // Jacobi eigenvectors
  double Q[TMAX * LQ];   // orthonormal block (rows >= T, cols >= k kept zero)
  double Y[TMAX * LQ];   // R Q, or the canonical U
  double red[NT];
  double rot_c[TMAX / 2 + 1], rot_s[TMAX / 2 + 1];
  int rot_p[TMAX / 2 + 1], rot_q[TMAX / 2 + 1];
  int perm[TMAX];
  int flag;
  int ok;
};

__device__ __forceinline__ double block_sum(double v, double* /*red*/) {
  return wave_reduce(v, [](double a, double b) { return a + b; });
}

__device__ __forceinline__ double block_max(double v, double* /*red*/) {
  return wave_reduce(v, [](double a, double b) { return fmax(a, b); });
}

// Products on the FP64 matrix cores (v_mfma_f64_16x16x4f64).  Operand
// layouts: lane l holds A[l%16][l/16] and B[l/16][l%16]; result element
// (4*r + l/16, l%16) is component r of lane l.  Every product below runs its
// whole contraction unrolled (operands zero padded to TMAX rows / KR columns),
// with one accumulator per output tile so that consecutive MFMAs are
// independent.
__device__ __forceinline__ d4 mfma64(double a, double b, d4 acc) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
}

// Y = R Q (T x k; rows >= T and columns >= k come out zero).
template <int KR, int TMAX, int KMAX>
__device__ __forceinline__ void mm_RQ(OiSmem<TMAX, KMAX>& s) {
  constexpr int TI = TMAX / 16, TJ = KR / 16;
  const int lane = threadIdx.x, r16 = lane % 16, q4 = lane / 16;
  d4 acc[TI][TJ];
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int kk = 0; kk < TMAX; kk += 4) {
    double b[TJ];
#pragma unroll
    for (int j = 0; j < TJ; ++j) b[j] = s.Q[(kk + q4) * s.LQ + j * 16 + r16];
#pragma unroll
    for (int i = 0; i < TI; ++i) {
      const double a = s.R[(i * 16 + r16) * s.LR + kk + q4];
#pragma unroll
      for (int j = 0; j < TJ; ++j) acc[i][j] = mfma64(a, b[j], acc[i][j]);
    }
  }
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) s.Y[(i * 16 + 4 * r + q4) * s.LQ + j * 16 + r16] = acc[i][j][r];
  __syncthreads();
}

// Y = R Q with bfloat16 operands and float32 accumulation (precision form):
// v_mfma_f32_16x16x32_bf16, lane l supplies A[l%16][8(l/16) .. +7] and
// B[8(l/16) .. +7][l%16]; component r of lane l is D[4(l/16) + r][l%16].
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <int KR, int TMAX, int KMAX>
__device__ __forceinline__ void mm_RQ_bf16(OiSmem<TMAX, KMAX>& s) {
  constexpr int TI = TMAX / 16, TJ = KR / 16;
  const int lane = threadIdx.x, r16 = lane % 16, q4 = lane / 16;
  f4 acc[TI][TJ];
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int kk = 0; kk < TMAX; kk += 32) {
    bf8 b[TJ];
#pragma unroll
    for (int j = 0; j < TJ; ++j)
#pragma unroll
      for (int e = 0; e < 8; ++e) b[j][e] = (__bf16)s.Q[(kk + 8 * q4 + e) * s.LQ + j * 16 + r16];
#pragma unroll
    for (int i = 0; i < TI; ++i) {
      bf8 a;
#pragma unroll
      for (int e = 0; e < 8; ++e) a[e] = (__bf16)s.R[(i * 16 + r16) * s.LR + kk + 8 * q4 + e];
#pragma unroll
      for (int j = 0; j < TJ; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[j], acc[i][j], 0, 0, 0);
    }
  }
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) s.Y[(i * 16 + 4 * q4 + r) * s.LQ + j * 16 + r16] = (double)acc[i][j][r];
  __syncthreads();
}

// A[0:KR, 0:KR] = X^T Z for T x KR blocks X, Z in LDS (stride LQ, rows >= T
// zero).  X == Z gives the Gram matrix.
template <int KR, int TMAX, int KMAX>
__device__ __forceinline__ void mm_XtZ(OiSmem<TMAX, KMAX>& s, const double* X, const double* Z) {
  constexpr int TN = KR / 16;
  const int lane = threadIdx.x, r16 = lane % 16, q4 = lane / 16;
  d4 acc[TN][TN];
#pragma unroll
  for (int i = 0; i < TN; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int kk = 0; kk < TMAX; kk += 4) {
    double a[TN], b[TN];
#pragma unroll
    for (int i = 0; i < TN; ++i) {
      a[i] = X[(kk + q4) * s.LQ + i * 16 + r16];
      b[i] = Z[(kk + q4) * s.LQ + i * 16 + r16];
    }
#pragma unroll
    for (int i = 0; i < TN; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j) acc[i][j] = mfma64(a[i], b[j], acc[i][j]);
  }
#pragma unroll
  for (int i = 0; i < TN; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) s.A[(i * 16 + 4 * r + q4) * s.LR + j * 16 + r16] = acc[i][j][r];
  __syncthreads();
}

// 1 / sqrt(d) for a normal d > 0: the hardware estimate refined by two
// Newton steps r <- r + r (1 - d r^2) / 2 (each roughly squares the relative
// error), a short dependent chain beside a rounded square root and division.
__device__ __forceinline__ double rsqrt_f64(double d) {
  double r = __builtin_amdgcn_rsq(d);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double e = fma(-d * r, r, 1.0);
    r = fma(0.5 * e, r, r);
  }
  return r;
}

// One pass of Cholesky QR in registers.  Lane i < KR holds row i of the KR x
// KR Gram matrix in g (identity rows/columns beyond k), lane t holds row t of
// the block in x (zero beyond column k and beyond row T).  Column j of the
// Cholesky factor L is formed at step j and broadcast by lane reads; it serves
// both the trailing update of g and the forward substitution x <- x L^-T,
// which proceed column by column together.  A pivot <= thresh fails the pass
// (returned false; the results are then discarded).
template <int KR>
__device__ __forceinline__ bool chol_qr_regs(double (&g)[KR], double (&x)[KR], double thresh) {
  const int lane = threadIdx.x;
  bool ok = true;
#pragma unroll
  for (int j = 0; j < KR; ++j) {
    const double d = readlane_f64(g[j], j);
    const bool good = d > thresh;
    ok = ok && good;
    const double inv = good ? rsqrt_f64(d) : 1.0;
    const double ljj = good ? d * inv : 1.0;
    const double lij = lane > j ? g[j] * inv : (lane == j ? ljj : 0.0);
    g[j] = lij;
    const double qj = x[j] * inv;
    x[j] = qj;
#pragma unroll
    for (int l = j + 1; l < KR; ++l) {
      const double c = readlane_f64(lij, l);  // L[l][j]
      g[l] = fma(-lij, c, g[l]);
      x[l] = fma(-qj, c, x[l]);
    }
  }
  return ok;
}

// The same pass for T <= 32 with both operands in one array: lanes 0..31 hold
// the rows of the block, lane 32 + i row i of the Gram matrix.  One FMA per
// entry and step serves both the trailing update and the substitution.
template <int KR>
__device__ __forceinline__ bool chol_qr_packed(double (&v)[KR], double thresh) {
  const int lane = threadIdx.x;
  const bool isG = lane >= 32;
  const int i = lane - 32;
  bool ok = true;
#pragma unroll
  for (int j = 0; j < KR; ++j) {
    const double d = readlane_f64(v[j], 32 + j);
    const bool good = d > thresh;
    ok = ok && good;
    const double inv = good ? rsqrt_f64(d) : 1.0;
    const double ljj = good ? d * inv : 1.0;
    const double own = isG ? (i > j ? v[j] * inv : (i == j ? ljj : 0.0)) : v[j] * inv;
    v[j] = own;
#pragma unroll
    for (int l = j + 1; l < KR; ++l) v[l] = fma(-own, readlane_f64(own, 32 + l), v[l]);
  }
  return ok;
}

// Gram-Schmidt in place on the block in s.Q (lane t < T works on row t):
// each column orthogonalised twice against the previous ones, four at a time
// (the four projections of a group are taken from the same vector, so their
// wavefront sums are in flight together; the groups follow one another, as
// in modified Gram-Schmidt); a column with no component left (below 1e-10 of
// its norm) is replaced by the identity direction e_m with the largest part
// outside the span found so far (first such m), then orthogonalised the same
// way.  Columns k..KMAX-1 are set to zero.  The fallback of `orthonormalise`
// for numerically rank-deficient blocks; its loops over columns stay rolled
// (short code).
template <int TMAX, int KMAX>
__device__ __forceinline__ void mgs_lds(OiSmem<TMAX, KMAX>& s, int T, int k) {
  constexpr int G = 4;  // projections per group
  static_assert(KMAX % G == 0, "column groups must not run past the block");
  const int lane = threadIdx.x;
  const bool row = lane < T;
  double* q = s.Q + (row ? lane : 0) * s.LQ;
  __syncthreads();
#pragma unroll 1
  for (int j = 0; j < k; ++j) {
    double v = row ? q[j] : 0.0;
    const double n0 = sqrt(block_sum(v * v, nullptr));
    double nj = 0.0;
#pragma unroll 1
    for (int attempt = 0; attempt < 2; ++attempt) {
      if (attempt == 1) {
        // completion: the identity direction with the largest part left
        double out = 1.0;
#pragma unroll 1
        for (int l = 0; l < j; ++l) out -= row ? q[l] * q[l] : 0.0;
        const double best = block_max(row ? out : -1.0, nullptr);
        const unsigned long long hit = __ballot(row && out == best);
        const int bm = hit ? __ffsll(hit) - 1 : 0;
        v = lane == bm ? 1.0 : 0.0;
      }
#pragma unroll 1
      for (int pass = 0; pass < 2; ++pass) {
#pragma unroll 1
        for (int l0 = 0; l0 < j; l0 += G) {
          double ql[G], d[G];
#pragma unroll
          for (int u = 0; u < G; ++u) {
            const double x = q[l0 + u];  // inside the row (KMAX % G == 0)
            ql[u] = (row && l0 + u < j) ? x : 0.0;
            d[u] = ql[u] * v;
          }
          wave_sum_n<G>(d);
#pragma unroll
          for (int u = 0; u < G; ++u) v = fma(-d[u], ql[u], v);
        }
      }
      nj = sqrt(block_sum(v * v, nullptr));
      if (attempt == 0 && (nj > 1e-10 * n0) && n0 != 0.0) break;
    }
    if (row) q[j] = v / nj;
  }
  if (row)
    for (int j = k; j < KMAX; ++j) q[j] = 0.0;
  __syncthreads();
}

// Q = orthonormal basis of span(X) (X = Y or Q, T x k), left in s.Q.
// Cholesky QR2 on the column-scaled block (columns of R Q differ in norm by
// the eigenvalue spread; scaling by the Gram diagonal removes that without
// changing the Q factor).  A pivot breakdown switches to shifted Cholesky QR3
// (Fukaya et al.: shift 11 (T k + k (k + 1)) u ||X||_F^2); `shifted` starts
// with the shifted pass directly (blocks R Q whose columns are known to be
// nearly dependent).  A breakdown after that, or an exactly zero column,
// switches to Gram-Schmidt with completion.  Returns the number of repairs
// (0: plain Cholesky QR2).
template <int KR, int TMAX, int KMAX>
__device__ __forceinline__ int orthonormalise(OiSmem<TMAX, KMAX>& s, const double* X, int T, int k,
                                              bool shifted = false) {
  const int lane = threadIdx.x;
  constexpr double thresh = 1e-15;  // pivots relative to the unit diagonal
  constexpr bool packed = TMAX <= 32;
  mm_XtZ<KR>(s, X, X);
  // column scales: lane r < k holds 1 / ||x_r|| (packed: lanes 32 + r too)
  const int r = packed ? (lane & 31) : lane;
  const double grr = r < k ? s.A[r * s.LR + r] : 1.0;
  const bool zero_col = __any(r < k && !(grr > 0.0));
  const double dinv = (r < k && grr > 0.0) ? 1.0 / sqrt(grr) : 1.0;
  double x[KR];
  double g[packed ? 1 : KR];
  // rows of the block (lanes < T; packed: lanes < 32) and of the Gram matrix
  // in A (packed: lane 32 + i holds row i; else lane i in g), both scaled
  // by the column scales when `scaled`; the block rows are reloaded from X
  // unless `gram_only`
  auto load = [&](bool scaled, bool gram_only) {
#pragma unroll
    for (int j = 0; j < KR; ++j) {
      const double dj = scaled ? readlane_f64(dinv, j) : 1.0;
      const double di = scaled ? dinv : 1.0;
      const int gi = packed ? lane - 32 : lane;
      const double gv = (gi >= 0 && gi < k) ? s.A[gi * s.LR + j] * di * dj
                                            : ((gi >= k && gi == j) ? 1.0 : 0.0);
      const double xv = lane < T ? X[lane * s.LQ + j] * dj : 0.0;
      if constexpr (packed) {
        x[j] = lane >= 32 ? gv : (gram_only ? x[j] : xv);
      } else {
        g[j] = gv;
        if (!gram_only) x[j] = xv;
      }
    }
  };
  auto pass = [&]() -> bool {
    if constexpr (packed)
      return chol_qr_packed<KR>(x, thresh);
    else
      return chol_qr_regs<KR>(g, x, thresh);
  };
  auto to_Q = [&]() {  // block rows back to s.Q (X may alias it)
    __syncthreads();
    if (lane < T && (!packed || lane < 32)) {
#pragma unroll
      for (int j = 0; j < KR; ++j) s.Q[lane * s.LQ + j] = x[j];
    }
    __syncthreads();
  };
  auto add_shift = [&]() {
    const double shift = 11.0 * (double)(T * k + k * (k + 1)) * 1.1102230246251565e-16 * (double)k;
#pragma unroll
    for (int j = 0; j < KR; ++j) {
      if constexpr (packed)
        x[j] += (lane - 32 == j && j < k) ? shift : 0.0;
      else
        g[j] += (lane == j && j < k) ? shift : 0.0;
    }
  };
  if (zero_col) {
    load(true, false);
    to_Q();
    mgs_lds(s, T, k);
    return 1;
  }
  // pass 0 factors the scaled X (shifted: with the shift, and three passes in
  // all); a breakdown of an unshifted pass 0 restarts it shifted; passes >= 1
  // factor the Gram matrix of the previous pass's Q
  int repairs = shifted ? 1 : 0, passes = shifted ? 3 : 2;
  bool shift = shifted;
#pragma unroll 1
  for (int p = 0; p < passes; ++p) {
    if (p > 0) {
      to_Q();
      mm_XtZ<KR>(s, s.Q, s.Q);
    }
    load(p == 0, p > 0);
    if (p == 0 && shift) add_shift();
    if (!pass()) {
      if (p == 0 && !shift) {  // restart shifted
        shift = true;
        repairs = 1;
        passes = 3;
        p = -1;
        continue;
      }
      if (p == 0) {  // the scaled X to s.Q for Gram-Schmidt
        load(true, false);
        to_Q();
        mgs_lds(s, T, k);
        return 2;
      }
      mgs_lds(s, T, k);  // s.Q still holds the last block
      return repairs + 2;
    }
  }
  to_Q();
  return repairs;
}

// Parallel cyclic Jacobi on the m x m symmetric matrix in A (round-robin
// pairing, every pair zeroed once per sweep); eigenvectors accumulate in V.
// A pair is skipped when |A_pq| <= max(eps sqrt(|A_pp A_qq|), eps ||A||_F)
// (below one ulp of the matrix a rotation changes nothing the matrix
// determines); stops after a sweep with no rotation.  General-size version,
// with the matrices in LDS (used for m > 32).  In each round the rotations
// are disjoint, so A J and V J are done by rows (thread x owns row x and
// updates its entries in columns p, q of every pair) and J^T (A J) by columns
// (thread y owns column y); the pairs go in batches of eight, each thread
// issuing all loads of a batch before its stores, so the LDS latency is paid
// once per batch.
template <int TMAX, int KMAX>
__device__ __forceinline__ void jacobi(OiSmem<TMAX, KMAX>& s, int m) {
  const int LR = s.LR;
  for (int e = threadIdx.x; e < m * m; e += NT)
    s.V[(e / m) * LR + e % m] = (e / m == e % m) ? 1.0 : 0.0;
  __syncthreads();
  if (m < 2) {
    if (threadIdx.x == 0) s.perm[0] = 0;
    __syncthreads();
    return;
  }
  const int me = m + (m & 1);
  const int np = me / 2;
  const double eps = 2.220446049250313e-16;
  double fro = 0.0;
  for (int e = threadIdx.x; e < m * m; e += NT) {
    const double v = s.A[(e / m) * LR + e % m];
    fro += v * v;
  }
  const double floor_abs = eps * sqrt(block_sum(fro, s.red));
  for (int sweep = 0; sweep < 60; ++sweep) {
    if (threadIdx.x == 0) s.flag = 0;
    __syncthreads();
    for (int round = 0; round < me - 1; ++round) {
      if (threadIdx.x < np) {
        const int i = threadIdx.x;
        int a, b;
        if (i == 0) {
          a = me - 1;
          b = round;
        } else {
          a = (round + i) % (me - 1);
          b = (round - i + me - 1) % (me - 1);
        }
        const int p = a < b ? a : b, q = a < b ? b : a;
        double c = 1.0, sn = 0.0;
        if (q < m) {
          const double apq = s.A[p * LR + q];
          const double app = s.A[p * LR + p], aqq = s.A[q * LR + q];
          if (fabs(apq) > fmax(eps * sqrt(fabs(app * aqq)), floor_abs) && apq != 0.0) {
            const double th = (aqq - app) / (2.0 * apq);
            const double t = copysign(1.0, th) / (fabs(th) + sqrt(th * th + 1.0));
            c = 1.0 / sqrt(t * t + 1.0);
            sn = t * c;
            s.flag = 1;
          }
        }
        s.rot_p[i] = p;
        s.rot_q[i] = q < m ? q : p;
        s.rot_c[i] = c;
        s.rot_s[i] = sn;
      }
      __syncthreads();
      // A <- A J and V <- V J: thread x owns row x; the pairs go in batches
      // of JB, every load of a batch issued before its stores
      constexpr int JB = 8;
      const int x = threadIdx.x;
      if (x < m) {
        for (int i0 = 0; i0 < np; i0 += JB) {
          double ap[JB], aq[JB], vp[JB], vq[JB], cc[JB], ss[JB];
          int pp[JB], qq[JB];
#pragma unroll
          for (int u = 0; u < JB; ++u) {
            const int i = i0 + u < np ? i0 + u : np - 1;
            pp[u] = s.rot_p[i];
            qq[u] = s.rot_q[i];
            cc[u] = s.rot_c[i];
            ss[u] = i0 + u < np ? s.rot_s[i] : 0.0;
            ap[u] = s.A[x * LR + pp[u]];
            aq[u] = s.A[x * LR + qq[u]];
            vp[u] = s.V[x * LR + pp[u]];
            vq[u] = s.V[x * LR + qq[u]];
          }
#pragma unroll
          for (int u = 0; u < JB; ++u) {
            if (ss[u] == 0.0) continue;
            const double c = cc[u], sn = ss[u];
            s.A[x * LR + pp[u]] = c * ap[u] - sn * aq[u];
            s.A[x * LR + qq[u]] = sn * ap[u] + c * aq[u];
            s.V[x * LR + pp[u]] = c * vp[u] - sn * vq[u];
            s.V[x * LR + qq[u]] = sn * vp[u] + c * vq[u];
          }
        }
      }
      __syncthreads();
      // A <- J^T A: thread y owns column y; the rotated pair's own
      // off-diagonal entries become zero
      const int y = threadIdx.x;
      if (y < m) {
        for (int i0 = 0; i0 < np; i0 += JB) {
          double rp[JB], rq[JB], cc[JB], ss[JB];
          int pp[JB], qq[JB];
#pragma unroll
          for (int u = 0; u < JB; ++u) {
            const int i = i0 + u < np ? i0 + u : np - 1;
            pp[u] = s.rot_p[i];
            qq[u] = s.rot_q[i];
            cc[u] = s.rot_c[i];
            ss[u] = i0 + u < np ? s.rot_s[i] : 0.0;
            rp[u] = s.A[pp[u] * LR + y];
            rq[u] = s.A[qq[u] * LR + y];
          }
#pragma unroll
          for (int u = 0; u < JB; ++u) {
            if (ss[u] == 0.0) continue;
            const double c = cc[u], sn = ss[u];
            s.A[pp[u] * LR + y] = (y == qq[u]) ? 0.0 : c * rp[u] - sn * rq[u];
            s.A[qq[u] * LR + y] = (y == pp[u]) ? 0.0 : sn * rp[u] + c * rq[u];
          }
        }
      }
      __syncthreads();
    }
    if (s.flag == 0) break;
    __syncthreads();
  }
  // order by eigenvalue, largest first (ties: lower index first)
  for (int i = threadIdx.x; i < m; i += NT) {
    const double li = s.A[i * LR + i];
    int rank = 0;
    for (int j = 0; j < m; ++j) {
      const double lj = s.A[j * LR + j];
      rank += (lj > li || (lj == li && j < i)) ? 1 : 0;
    }
    s.perm[rank] = i;
  }
  __syncthreads();
}


// Register-resident parallel cyclic Jacobi for m <= M (M = 16 or 32, zero
// padded to M; padding is never rotated because its off-diagonal entries are
// exactly zero).  Lane l < 32 holds row l of A, lane 32 + l row l of V; all
// register indices are constants.  Pairing by the circle method: in every
// round the slots (k, M - 1 - k) are rotated together, then slot 0 stays and
// the contents of slots 1..M-1 move one place along a ring (columns: register
// moves; rows of A: one lane shuffle per entry).  After M - 1 rounds every
// pair has met once and the slots are back in their original order.
// Skip rule and ordering as in `jacobi`.
template <int M, int TMAX, int KMAX>
__device__ __forceinline__ void jacobi_regs(OiSmem<TMAX, KMAX>& s, int m) {
  const int LR = s.LR;
  const int lane = threadIdx.x;
  const int t = lane & 31;
  const bool isA = lane < 32;
  const bool rowA = isA && t < M;
  double a[M];
  double fro = 0.0;
#pragma unroll
  for (int j = 0; j < M; ++j) {
    const double v = (t < m && j < m) ? s.A[t * LR + j] : 0.0;
    a[j] = isA ? v : (t == j ? 1.0 : 0.0);
    fro += isA ? v * v : 0.0;
  }
  const double eps = 2.220446049250313e-16;
  const double floor_abs = eps * sqrt(block_sum(fro, s.red));
  const int partner = M - 1 - t;               // pair (t, M - 1 - t)
  const int pair = t < partner ? t : partner;  // pair index
  const bool is_p = t < partner;
  __syncthreads();
  int sweeps_done = 0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    bool rotated = false;
    for (int round = 0; round < M - 1; ++round) {
      // this lane's diagonal and off-diagonal entry with its partner
      double diag = 0.0, off = 0.0;
#pragma unroll
      for (int j = 0; j < M; ++j) {
        diag = (j == t) ? a[j] : diag;
        off = (j == partner) ? a[j] : off;
      }
      const double dpart = M == 16 ? dpp_f64<kDppRowMirror>(diag) : shfl_f64(diag, partner);
      const double app = is_p ? diag : dpart, aqq = is_p ? dpart : diag;
      // the rotation of each pair is decided and computed by its p row only
      double c = 1.0, sn = 0.0;
      if (rowA && is_p && fabs(off) > fmax(eps * sqrt(fabs(app * aqq)), floor_abs) && off != 0.0) {
        const double th = (aqq - app) / (2.0 * off);
        const double tt = copysign(1.0, th) / (fabs(th) + sqrt(th * th + 1.0));
        c = 1.0 / sqrt(tt * tt + 1.0);
        sn = tt * c;
      }
      const bool any = __any(sn != 0.0);
      rotated = rotated || any;
      if (any) {
        if (rowA && is_p) {
          s.rot_c[pair] = c;
          s.rot_s[pair] = sn;
        }
        __syncthreads();
        // A <- A J and V <- V J: lane-local on its row
#pragma unroll
        for (int i = 0; i < M / 2; ++i) {
          const double ci = s.rot_c[i], si = s.rot_s[i];
          const double xp = a[i], xq = a[M - 1 - i];
          a[i] = ci * xp - si * xq;
          a[M - 1 - i] = si * xp + ci * xq;
        }
        // A <- J^T A: rows p and q combine (partner's row by lane exchange),
        // both with the rotation of their pair
        if (rowA) {
          c = s.rot_c[pair];
          sn = s.rot_s[pair];
        }
        const bool upd = rowA && sn != 0.0;
#pragma unroll
        for (int j = 0; j < M; ++j) {
          const double pj = M == 16 ? dpp_f64<kDppRowMirror>(a[j]) : shfl_f64(a[j], partner);
          const double v = is_p ? c * a[j] - sn * pj : sn * pj + c * a[j];
          a[j] = upd ? ((j == partner) ? 0.0 : v) : a[j];
        }
        __syncthreads();
      }
      // ring move of the slots: columns (all lanes) and rows (A lanes)
      {
        const double last = a[M - 1];
#pragma unroll
        for (int j = M - 1; j >= 2; --j) a[j] = a[j - 1];
        a[1] = last;
      }
      // rows: lane t takes lane t - 1's row (t >= 2), lane 1 takes lane
      // M - 1's, lane 0 keeps its own
#pragma unroll
      for (int j = 0; j < M; ++j) {
        const double sh = dpp_f64<kDppWaveRor1>(a[j]);
        const double last = readlane_f64(a[j], M - 1);
        a[j] = rowA ? (t == 0 ? a[j] : (t == 1 ? last : sh)) : a[j];
      }
    }
    sweeps_done = sweep + 1;
    if (!rotated) break;
    // The slots are back in their original order.  If every pair already
    // passes the skip test (checked from both rows, so never looser than the
    // test of a round), the next sweep would rotate nothing: stop here.
    bool pending = false;
    double dtt = 0.0;
#pragma unroll
    for (int i = 0; i < M; ++i) dtt = (i == t) ? a[i] : dtt;
#pragma unroll
    for (int j = 0; j < M; ++j) {
      const double djj = readlane_f64(a[j], j);
      const double x = a[j];
      pending = pending || (rowA && j != t && x != 0.0 &&
                            fabs(x) > fmax(eps * sqrt(fabs(dtt * djj)), floor_abs));
    }
    if (!__any(pending)) break;
  }
  if (threadIdx.x == 0) s.flag = sweeps_done;  // sweeps used (for inspection)
  // write back: diagonal of A, rows of V
#pragma unroll
  for (int j = 0; j < M; ++j) {
    if (isA && t < m && j == t) s.A[t * LR + t] = a[j];
    if (!isA && t < m && j < m) s.V[t * LR + j] = a[j];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < m; i += NT) {
    const double li = s.A[i * LR + i];
    int rank = 0;
    for (int j = 0; j < m; ++j) {
      const double lj = s.A[j * LR + j];
      rank += (lj > li || (lj == li && j < i)) ? 1 : 0;
    }
    s.perm[rank] = i;
  }
  __syncthreads();
}

// Value of v held by lane (t ^ R) of the same 16-lane row, for lane t of the
// row (R < 16): one DPP move for R = 1, 2, 3 (quad_perm), 7 (row_half_mirror:
// t -> 7 - t within eight lanes), 8 (row_ror by 8) and 15 (row_mirror), two
// moves for the other values (R = a ^ b with a in {7, 8, 15}, b in {1, 2, 3}).
template <int R>
__device__ __forceinline__ double xor16(double v) {
  if constexpr (R == 0) return v;
  else if constexpr (R == 1) return dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
  else if constexpr (R == 2) return dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
  else if constexpr (R == 3) return dpp_f64<0x1B>(v);   // quad_perm [3,2,1,0]
  else if constexpr (R == 7) return dpp_f64<0x141>(v);  // row_half_mirror
  else if constexpr (R == 8) return dpp_f64<0x128>(v);  // row_ror:8
  else if constexpr (R == 15) return dpp_f64<kDppRowMirror>(v);
  else if constexpr (R < 7) return xor16<7>(xor16<(R ^ 7)>(v));
  else if constexpr (R < 12) return xor16<8>(xor16<(R ^ 8)>(v));
  else return xor16<15>(xor16<(R ^ 15)>(v));
}

// One round of `jacobi_xor16`: every pair (t, t ^ R) is rotated together.
// Registers hold rows XOR-permuted (b[j] = row entry at column t ^ j), so the
// diagonal is b[0] and the pair's off-diagonal entry is b[R] on every lane.
// Both lanes of a pair compute the same rotation from the p row's A_pq (p the
// lower index); a lane keeps c and its signed sine (+s on p, -s on q).
template <int R>
__device__ __forceinline__ void jacobi_xor_round(double (&b)[16], int t, bool rowA, bool rowV,
                                                 double floor_abs, bool& rotated) {
  constexpr int HB = R >= 8 ? 8 : R >= 4 ? 4 : R >= 2 ? 2 : 1;  // highest bit of R
  constexpr double eps2 = 2.220446049250313e-16 * 2.220446049250313e-16;
  const bool is_p = (t & HB) == 0;
  const double d = b[0], off = b[R];
  const double dq = xor16<R>(d), offq = xor16<R>(off);
  const double app = is_p ? d : dq, aqq = is_p ? dq : d, apq = is_p ? off : offq;
  const bool rot = rowA && apq != 0.0 && fabs(apq) > floor_abs && apq * apq > eps2 * fabs(app * aqq);
  if (!__any(rot)) return;
  rotated = true;
  double c = 1.0, sg = 0.0, dnew = d;
  if (rot) {
    // tan of the angle that zeroes A_pq: 2 A_pq sign(z) / (|z| + sqrt(z^2 + 4 A_pq^2)),
    // z = A_qq - A_pp (the usual form, scaled by 2 |A_pq|)
    const double z = aqq - app;
    const double tn = 2.0 * apq * copysign(1.0, z) / (fabs(z) + sqrt(z * z + 4.0 * apq * apq));
    c = 1.0 / sqrt(tn * tn + 1.0);
    sg = is_p ? tn * c : -(tn * c);
    dnew = is_p ? app - tn * apq : aqq + tn * apq;
  }
  // the rows of V (lanes 16..31) take the rotations of the A rows (lanes 0..15)
  const double cs = swap16_f64(c), ss = swap16_f64(sg);
  const double ccol = rowV ? cs : c, scol = rowV ? ss : sg;
  // A <- A J, V <- V J: register j (column x = t ^ j) pairs with j ^ R; the
  // rotation of column x's pair sits on lane x, i.e. t ^ j
  auto col_pair = [&](auto jc) {
    constexpr int j = decltype(jc)::value;
    if constexpr ((j & HB) == 0) {
      const double cj = xor16<j>(ccol), sj = xor16<j>(scol);
      const double x = b[j], y = b[j ^ R];
      b[j] = cj * x - sj * y;
      b[j ^ R] = cj * y + sj * x;
    }
  };
  col_pair(std::integral_constant<int, 0>{});
  col_pair(std::integral_constant<int, 1>{});
  col_pair(std::integral_constant<int, 2>{});
  col_pair(std::integral_constant<int, 3>{});
  col_pair(std::integral_constant<int, 4>{});
  col_pair(std::integral_constant<int, 5>{});
  col_pair(std::integral_constant<int, 6>{});
  col_pair(std::integral_constant<int, 7>{});
  col_pair(std::integral_constant<int, 8>{});
  col_pair(std::integral_constant<int, 9>{});
  col_pair(std::integral_constant<int, 10>{});
  col_pair(std::integral_constant<int, 11>{});
  col_pair(std::integral_constant<int, 12>{});
  col_pair(std::integral_constant<int, 13>{});
  col_pair(std::integral_constant<int, 14>{});
  col_pair(std::integral_constant<int, 15>{});
  // A <- J^T A on the A rows: row t mixes with row t ^ R, whose entry at
  // column t ^ j is that lane's register j ^ R
  double pb[16];
  auto fetch = [&](auto jc) {
    constexpr int j = decltype(jc)::value;
    if constexpr (j != 0 && j != R) pb[j] = xor16<R>(b[j ^ R]);
  };
  fetch(std::integral_constant<int, 1>{});
  fetch(std::integral_constant<int, 2>{});
  fetch(std::integral_constant<int, 3>{});
  fetch(std::integral_constant<int, 4>{});
  fetch(std::integral_constant<int, 5>{});
  fetch(std::integral_constant<int, 6>{});
  fetch(std::integral_constant<int, 7>{});
  fetch(std::integral_constant<int, 8>{});
  fetch(std::integral_constant<int, 9>{});
  fetch(std::integral_constant<int, 10>{});
  fetch(std::integral_constant<int, 11>{});
  fetch(std::integral_constant<int, 12>{});
  fetch(std::integral_constant<int, 13>{});
  fetch(std::integral_constant<int, 14>{});
  fetch(std::integral_constant<int, 15>{});
  const double nsg = -sg;
#pragma unroll
  for (int j = 1; j < 16; ++j)
    if (j != R) b[j] = fma(c, b[j], nsg * pb[j]);
  // the pair's own entries: diagonal from the rotation formula, A_pq = 0
  b[0] = rot ? dnew : b[0];
  b[R] = rot ? 0.0 : b[R];
}

// Sweep-end test of `jacobi_xor16`: does any off-diagonal entry of an A row
// still fail the skip rule?  Each entry is tested on its own row, so every
// pair is tested from both of its rows.
template <int J>
__device__ __forceinline__ bool jacobi_xor_pending(const double (&b)[16], bool rowA,
                                                   double floor_abs) {
  if constexpr (J == 16) {
    return false;
  } else {
    constexpr double eps2 = 2.220446049250313e-16 * 2.220446049250313e-16;
    const double dj = xor16<J>(b[0]);
    const double x = b[J];
    const bool p = rowA && x != 0.0 && fabs(x) > floor_abs && x * x > eps2 * fabs(b[0] * dj);
    return p || jacobi_xor_pending<J + 1>(b, rowA, floor_abs);
  }
}

// Register-resident parallel cyclic Jacobi for m <= 16 with every row kept in
// its lane (zero padded to 16; padding is never rotated because its
// off-diagonal entries are exactly zero).  Round r = 1..15 rotates the pairs
// (t, t ^ r) together: the XOR one-factorisation of 16 indices, in which
// every pair meets exactly once per sweep and every partner exchange is a
// fixed DPP lane move.  Lane t < 16 holds row t of A, lane 16 + t row t of V,
// both XOR-permuted (register j holds column t ^ j).  The diagonal is carried
// by the rotation formulas (A'_pp = A_pp - tan A_pq, A'_qq = A_qq + tan A_pq)
// and the rotated pair entry is set to zero.  Skip rule as in `jacobi`, in
// squared form; stops after a sweep with no rotation or when no entry is
// left that a rotation would change.  Eigenvalue ordering as in `jacobi`.
template <int TMAX, int KMAX>
__device__ __forceinline__ void jacobi_xor16(OiSmem<TMAX, KMAX>& s, int m) {
  const int LR = s.LR;
  const int lane = threadIdx.x;
  const int t = lane & 15;
  const bool rowA = lane < 16, rowV = lane >= 16 && lane < 32;
  double b[16];
  double fro = 0.0;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int x = t ^ j;
    const double v = (rowA && t < m && x < m) ? s.A[t * LR + x] : 0.0;
    b[j] = rowA ? v : ((rowV && j == 0) ? 1.0 : 0.0);
    fro += v * v;
  }
  const double floor_abs = 2.220446049250313e-16 * sqrt(block_sum(fro, s.red));
  __syncthreads();
  int sweeps_done = 0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    bool rotated = false;
    jacobi_xor_round<1>(b, t, rowA, rowV, floor_abs, rotated);
    jacobi_xor_round<2>(b, t, rowA, rowV, floor_abs, rotated);
    jacobi_xor_round<3>(b, t, rowA, rowV, floor_abs, rotated);
    jacobi_xor_round<4>(b, t, rowA, rowV, floor_abs, rotated);
    jacobi_xor_round<5>(b, t, rowA, rowV, floor_abs, rotated);
    jacobi_xor_round<6>(b, t, rowA, rowV, floor_abs, rotated);
    jacobi_xor_round<7>(b, t, rowA, rowV, floor_abs, rotated);
    jacobi_xor_round<8>(b, t, rowA, rowV, floor_abs, rotated);
    jacobi_xor_round<9>(b, t, rowA, rowV, floor_abs, rotated);
    jacobi_xor_round<10>(b, t, rowA, rowV, floor_abs, rotated);
    jacobi_xor_round<11>(b, t, rowA, rowV, floor_abs, rotated);
    jacobi_xor_round<12>(b, t, rowA, rowV, floor_abs, rotated);
    jacobi_xor_round<13>(b, t, rowA, rowV, floor_abs, rotated);
    jacobi_xor_round<14>(b, t, rowA, rowV, floor_abs, rotated);
    jacobi_xor_round<15>(b, t, rowA, rowV, floor_abs, rotated);
    sweeps_done = sweep + 1;
    if (!rotated) break;
    if (!__any(jacobi_xor_pending<1>(b, rowA, floor_abs))) break;
  }
  if (threadIdx.x == 0) s.flag = sweeps_done;  // sweeps used (for inspection)
  // write back: diagonal of A, rows of V
  if (rowA && t < m) s.A[t * LR + t] = b[0];
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int x = t ^ j;
    if (rowV && t < m && x < m) s.V[t * LR + x] = b[j];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < m; i += NT) {
    const double li = s.A[i * LR + i];
    int rank = 0;
    for (int j = 0; j < m; ++j) {
      const double lj = s.A[j * LR + j];
      rank += (lj > li || (lj == li && j < i)) ? 1 : 0;
    }
    s.perm[rank] = i;
  }
  __syncthreads();
}

// Eigenvectors of the m x m symmetric matrix in A: register Jacobi up to
// m = 32, the LDS version above.  FAST16 (set for the Ritz step of the
// kernels for k <= 16, where the Ritz matrix always fits) selects the in-place
// XOR-schedule version; it is instantiated only there, as it is long code.
template <bool FAST16 = false, int TMAX, int KMAX>
__device__ __forceinline__ void eigen_sym(OiSmem<TMAX, KMAX>& s, int m) {
  if constexpr (FAST16) {
    if (m <= 16)
      jacobi_xor16(s, m);
    else
      jacobi(s, m);  // not reached from the k <= 16 kernels; short code
  } else {
    if (m <= 32)
      jacobi_regs<32>(s, m);
    else
      jacobi(s, m);
  }
}

// Sign rule on the T x k columns held in Y: the entry of largest magnitude
// (first one on a tie) becomes positive.
template <int TMAX, int KMAX>
__device__ __forceinline__ void sign_fix(OiSmem<TMAX, KMAX>& s, int T, int k) {
  for (int j = threadIdx.x; j < k; j += NT) {
    int im = 0;
    double vm = -1.0;
    for (int t = 0; t < T; ++t) {
      const double a = fabs(s.Y[t * s.LQ + j]);
      if (a > vm) {
        vm = a;
        im = t;
      }
    }
    if (s.Y[im * s.LQ + j] < 0.0)
      for (int t = 0; t < T; ++t) s.Y[t * s.LQ + j] = -s.Y[t * s.LQ + j];
  }
  __syncthreads();
}

// ||R Q - Q (Q^T R Q)||_F / ||R||_F with Y = R Q already computed; leaves
// H = Q^T Y (symmetrised) in A.  Both products on the matrix cores.
template <int KR, int TMAX, int KMAX>
__device__ __forceinline__ double residual_and_H(OiSmem<TMAX, KMAX>& s, int k, double normR) {
  mm_XtZ<KR>(s, s.Q, s.Y);
  constexpr int TI = TMAX / 16, TJ = KR / 16;
  const int lane = threadIdx.x, r16 = lane % 16, q4 = lane / 16;
  d4 acc[TI][TJ];
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int kk = 0; kk < KR; kk += 4) {
    double b[TJ];
#pragma unroll
    for (int j = 0; j < TJ; ++j) b[j] = s.A[(kk + q4) * s.LR + j * 16 + r16];
#pragma unroll
    for (int i = 0; i < TI; ++i) {
      const double a = s.Q[(i * 16 + r16) * s.LQ + kk + q4];
#pragma unroll
      for (int j = 0; j < TJ; ++j) acc[i][j] = mfma64(a, b[j], acc[i][j]);
    }
  }
  double ss = 0.0;
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double e = s.Y[(i * 16 + 4 * r + q4) * s.LQ + j * 16 + r16] - acc[i][j][r];
        ss = fma(e, e, ss);
      }
  const double res = block_sum(ss, s.red);
  __syncthreads();
  for (int e = threadIdx.x; e < k * k; e += NT) {
    const int a = e / k, b = e % k;
    if (b > a) {
      const double h = 0.5 * (s.A[a * s.LR + b] + s.A[b * s.LR + a]);
      s.A[a * s.LR + b] = h;
      s.A[b * s.LR + a] = h;
    }
  }
  __syncthreads();
  return normR > 0.0 ? sqrt(res) / normR : 0.0;
}

// Ritz vectors Y = Q V(:, perm) (columns in decreasing eigenvalue order).
template <int KR, int TMAX, int KMAX>
__device__ __forceinline__ void ritz_vectors(OiSmem<TMAX, KMAX>& s, int k) {
  constexpr int TI = TMAX / 16, TJ = KR / 16;
  const int lane = threadIdx.x, r16 = lane % 16, q4 = lane / 16;
  d4 acc[TI][TJ];
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int kk = 0; kk < KR; kk += 4) {
    double b[TJ];
#pragma unroll
    for (int j = 0; j < TJ; ++j) {
      const int col = j * 16 + r16, row = kk + q4;
      b[j] = (col < k && row < k) ? s.V[row * s.LR + s.perm[col]] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < TI; ++i) {
      const double a = s.Q[(i * 16 + r16) * s.LQ + kk + q4];
#pragma unroll
      for (int j = 0; j < TJ; ++j) acc[i][j] = mfma64(a, b[j], acc[i][j]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) s.Y[(i * 16 + 4 * r + q4) * s.LQ + j * 16 + r16] = acc[i][j][r];
  __syncthreads();
}

// Algorithm 1's iterations and the Ritz step: start block in Q (the previous
// window's U, or a caller-given block), sweeps Y = R Q, Q = QR(Y) until the
// residual test passes or the sweep cap, then U = Q V from H = Q^T R Q = V
// diag(mu) V^T; U is left in Y (not yet sign-fixed).
template <int KR, int TMAX, int KMAX>
__device__ __forceinline__ void oi_sweeps(OiSmem<TMAX, KMAX>& s, int T, int k, int max_sweeps, double tol,
                                          double normR, bool bf16, bool q_orthonormal, int& sweeps,
                                          int& repairs, double& resid, bool ritz = true) {
  // precision form: bfloat16 products until the stage tolerance (or one sweep
  // before the cap), then full-precision refinement sweeps (at least one)
  // until tol, or until a sweep no longer reduces the residual by a tenth
  // (the subspace has reached what the bfloat16 covariance determines)
  const double stage_tol = tol > DMC_BF16_STAGE_TOL ? tol : DMC_BF16_STAGE_TOL;
  bool refining = false;
  double prev = 0.0;
  // sweep 0 only orthonormalises the start (a start that is already
  // orthonormal, the previous window's U, is kept) and forms R Q; one code
  // path serves it and the sweeps, so the long orthonormalisation is
  // instantiated once
  for (int sw = 0; sw <= max_sweeps; ++sw) {
    // from the previous window's subspace, R Q spreads its columns by the
    // eigenvalue spread (nearly dependent after scaling): start shifted
    if (sw > 0 || !q_orthonormal)
      repairs += orthonormalise<KR>(s, sw == 0 ? s.Q : s.Y, T, k, sw > 0 && q_orthonormal) ? 1 : 0;
    if (bf16)
      mm_RQ_bf16<KR>(s);
    else
      mm_RQ<KR>(s);
    if (sw == 0) continue;
    sweeps = sw;
    resid = residual_and_H<KR>(s, k, normR);
    if (bf16) {
      if (resid <= stage_tol || sw + 1 >= max_sweeps) {
        bf16 = false;
        refining = true;
        prev = -1.0;
        mm_RQ<KR>(s);  // full-precision product for the refinement sweeps
      }
      continue;
    }
    if (resid <= tol) break;
    if (refining) {
      if (prev > 0.0 && resid > 0.9 * prev) break;
      prev = resid;
    }
  }
  if (ritz) {
    eigen_sym<KR == 16>(s, k);
    ritz_vectors<KR>(s, k);
  }
}

// Outputs of window w, coordinate c from the canonical U in s.Y: U in the
// frames' type (u_out) and in float64 (u_canon, which the dictionary coder
// reads).
template <int TMAX, int KMAX, typename Real>
__device__ __forceinline__ void oi_outputs(OiSmem<TMAX, KMAX>& s, const OiArgs& a, int w, int c) {
  const int T = a.T, k = a.k;
  Real* uo = a.u_out ? (Real*)a.u_out + ((size_t)w * a.ncoord + c) * T * k : nullptr;
  double* uc = a.u_canon ? a.u_canon + ((size_t)w * a.ncoord + c) * T * k : nullptr;
  for (int e = threadIdx.x; e < T * k; e += NT) {
    const double u = s.Y[(e / k) * s.LQ + e % k];
    if (uo) uo[e] = (Real)u;
    if (uc) uc[e] = u;
  }
}

// One workgroup (one wavefront) per coordinate; KR = k rounded up to the
// 16-column tile of the matrix-core products (16 or 32).
// The work of one workgroup: coordinate c of windows w_begin..w_end-1 (the
// whole chain for DMC_INIT_PREV, one window otherwise).
template <int TMAX, int KMAX, int KR, typename Real>
__device__ __forceinline__ void oi_run(OiSmem<TMAX, KMAX>& s, const OiArgs& a, int c, int w_begin,
                                       int w_end) {
  const int T = a.T, k = a.k;
  const int tid = threadIdx.x;
  const bool chain = a.init == DMC_INIT_PREV;
  for (int e = tid; e < TMAX * s.LQ; e += NT) {
    s.Q[e] = 0.0;
    s.Y[e] = 0.0;
  }
  __syncthreads();
  for (int w = w_begin; w < w_end; ++w) {
    // ---- load R_c of window w (zero padded), every load in flight at once ----
    const double* Rg = a.R + ((size_t)w * a.ncoord + c) * T * T;
    constexpr int PER = TMAX * TMAX / NT, CH = 16;  // 16 loads in flight per lane
    double part = 0.0;
    for (int u0 = 0; u0 < PER; u0 += CH) {
      double rv[CH];
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        const int e = tid + (u0 + u) * NT, i = e / TMAX, j = e % TMAX;
        rv[u] = (i < T && j < T) ? Rg[i * T + j] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        const int e = tid + (u0 + u) * NT, i = e / TMAX, j = e % TMAX;
        s.R[i * s.LR + j] = rv[u];
        part = fma(rv[u], rv[u], part);
      }
    }
    __syncthreads();
    const double normR = sqrt(block_sum(part, s.red));

    int sweeps = 0, repairs = 0;
    double resid = 0.0;
    bool defer = false;
    // exact start: always with DMC_INIT_EXACT, else for a missing start block
    // (window 0 of the chain; any window otherwise)
    const bool exact = a.init == DMC_INIT_EXACT ||
                       (a.init != DMC_INIT_LEARNED && a.q_start == nullptr && (w == 0 || !chain));
    if (exact) {
      // exact start of Algorithm 1: eigenvectors of R (Eq. 5)
      for (int e = tid; e < TMAX * s.LR; e += NT) s.A[e] = s.R[e];
      __syncthreads();
      eigen_sym(s, T);
      for (int e = tid; e < T * k; e += NT) {
        const int t = e / k, j = e % k;
        s.Y[t * s.LQ + j] = s.V[t * s.LR + s.perm[j]];
      }
      __syncthreads();
      sign_fix(s, T, k);
      for (int e = tid; e < T * k; e += NT) s.Q[(e / k) * s.LQ + e % k] = s.Y[(e / k) * s.LQ + e % k];
      __syncthreads();
      mm_RQ<KR>(s);
      resid = residual_and_H<KR>(s, k, normR);
      // canonical U = Q (already sorted and sign-fixed); keep it in Y
      for (int e = tid; e < T * k; e += NT) s.Y[(e / k) * s.LQ + e % k] = s.Q[(e / k) * s.LQ + e % k];
      __syncthreads();
    } else {
      if (!chain || w == 0) {
        // caller-given start (window 0 of the chain, or this window's own
        // block), or Omega for the sketch start R_c Omega
        constexpr int PQ = TMAX * KR / NT, CQ = PQ < 16 ? PQ : 16;
        // the network's prediction for this (window, coordinate), or the
        // caller's block
        const float* ql = a.init == DMC_INIT_LEARNED
                              ? a.q_learned + ((size_t)w * a.ncoord + c) * T * k
                              : nullptr;
        const Real* q0 = (const Real*)a.q_start;
        if (!ql) {
          if (a.init == DMC_INIT_RANDOM) q0 += ((size_t)w * a.ncoord + c) * T * k;
          else if (a.init != DMC_INIT_SKETCH) q0 += (size_t)c * T * k;
        }
        for (int u0 = 0; u0 < PQ; u0 += CQ) {
          double qv[CQ];
#pragma unroll
          for (int u = 0; u < CQ; ++u) {
            const int e = tid + (u0 + u) * NT;
            qv[u] = e < T * k ? (ql ? (double)ql[e] : (double)q0[e]) : 0.0;
          }
#pragma unroll
          for (int u = 0; u < CQ; ++u) {
            const int e = tid + (u0 + u) * NT;
            if (e < T * k) s.Q[(e / k) * s.LQ + e % k] = qv[u];
          }
        }
        __syncthreads();
        if (a.init == DMC_INIT_SKETCH) {
          mm_RQ<KR>(s);  // Y = R_c Omega
          for (int e = tid; e < T * k; e += NT) s.Q[(e / k) * s.LQ + e % k] = s.Y[(e / k) * s.LQ + e % k];
          __syncthreads();
        }
      }
      // chained windows with deferral: the Ritz step and the outputs run
      // afterwards for every window at once (k_oi_ritz), and the next window
      // starts from Q, which spans the same subspace as this window's U_k
      // (the sweeps, their residual test and the Ritz step depend on the
      // start's span only)
      defer = chain && a.ritz_qh != nullptr;
      oi_sweeps<KR>(s, T, k, a.max_sweeps, a.tol, normR, a.precision == DMC_BF16, chain && w > 0,
                    sweeps, repairs, resid, !defer);
      if (defer) {
        double* dst = a.ritz_qh + ((size_t)w * a.ncoord + c) * (T * k + k * k);
        for (int e = tid; e < T * k; e += NT) dst[e] = s.Q[(e / k) * s.LQ + e % k];
        for (int e = tid; e < k * k; e += NT) dst[T * k + e] = s.A[(e / k) * s.LR + e % k];
      } else {
        sign_fix(s, T, k);
      }
    }
    if (chain && a.ritz_flag && tid == 0) a.ritz_flag[w * a.ncoord + c] = defer ? 1 : 0;
    if (!defer) {
      oi_outputs<TMAX, KMAX, Real>(s, a, w, c);
      // the next window starts from this window's U_k
      for (int e = tid; e < T * k; e += NT) s.Q[(e / k) * s.LQ + e % k] = s.Y[(e / k) * s.LQ + e % k];
    }
    __syncthreads();
    if (tid == 0 && a.stats) {
      a.stats[w].sweeps[c] = sweeps;
      a.stats[w].shifts[c] = repairs;
      a.stats[w].resid[c] = resid;
    }
  }
}

// DMC_INIT_PREV chains the windows in one workgroup per coordinate; the other
// starts give every (window, coordinate) its own workgroup.
template <int TMAX, int KMAX, int KR, typename Real>
__global__ void __launch_bounds__(NT) k_oi(OiArgs a) {
  __shared__ OiSmem<TMAX, KMAX> s;
  const bool chain = a.init == DMC_INIT_PREV;
  const int w_begin = chain ? 0 : (int)blockIdx.y;
  oi_run<TMAX, KMAX, KR, Real>(s, a, blockIdx.x, w_begin, chain ? a.nw : w_begin + 1);
}

// The deferred Ritz step of the chained path (Algorithm 1 followed by Eq. 5 on
// the converged block): workgroup (c, w) takes window w's Q and H = Q^T R Q,
// forms the canonical U = Q V (eigenvectors of H, largest first, sign rule)
// and writes the window's outputs.  All windows run at once.
template <int TMAX, int KMAX, int KR, typename Real>
__global__ void __launch_bounds__(NT) k_oi_ritz(OiArgs a) {
  __shared__ OiSmem<TMAX, KMAX> s;
  const int c = blockIdx.x, w = blockIdx.y;
  if (a.ritz_flag[w * a.ncoord + c] == 0) return;  // whole workgroup: handled by k_oi
  const int T = a.T, k = a.k, tid = threadIdx.x;
  const double* src = a.ritz_qh + ((size_t)w * a.ncoord + c) * (T * k + k * k);
  for (int e = tid; e < TMAX * s.LQ; e += NT) s.Q[e] = 0.0;
  __syncthreads();
  for (int e = tid; e < T * k; e += NT) s.Q[(e / k) * s.LQ + e % k] = src[e];
  for (int e = tid; e < k * k; e += NT) s.A[(e / k) * s.LR + e % k] = src[T * k + e];
  __syncthreads();
  eigen_sym<KR == 16>(s, k);
  ritz_vectors<KR>(s, k);
  sign_fix(s, T, k);
  oi_outputs<TMAX, KMAX, Real>(s, a, w, c);
}

// Many sequences in one launch: workgroup b runs job jobs[b] = (sequence,
// first window, end window, coordinate) of args[sequence].
template <int TMAX, int KMAX, int KR, typename Real>
__global__ void __launch_bounds__(NT) k_oi_batch(const OiArgs* __restrict__ args,
                                                 const int4* __restrict__ jobs) {
  __shared__ OiSmem<TMAX, KMAX> s;
  const int4 j = jobs[blockIdx.x];
  const OiArgs a = args[j.x];
  oi_run<TMAX, KMAX, KR, Real>(s, a, j.w, j.y, j.z);
}

}  // namespace

template <int TMAX, int KR>
void launch_oi_t(hipStream_t st, const OiArgs& a) {
  const dim3 grid(a.ncoord, a.init == DMC_INIT_PREV ? 1 : a.nw);
  const bool deferred = a.init == DMC_INIT_PREV && a.ritz_qh != nullptr;
  if (a.precision == DMC_FP64) {
    hipLaunchKernelGGL((k_oi<TMAX, 32, KR, double>), grid, dim3(NT), 0, st, a);
    if (deferred)
      hipLaunchKernelGGL((k_oi_ritz<TMAX, 32, KR, double>), dim3(a.ncoord, a.nw), dim3(NT), 0, st, a);
  } else {
    hipLaunchKernelGGL((k_oi<TMAX, 32, KR, float>), grid, dim3(NT), 0, st, a);
    if (deferred)
      hipLaunchKernelGGL((k_oi_ritz<TMAX, 32, KR, float>), dim3(a.ncoord, a.nw), dim3(NT), 0, st, a);
  }
}

template <int TMAX, int KR>
void launch_oi_batch_t(hipStream_t st, int precision, const OiArgs* args, const int4* jobs,
                       int njobs) {
  if (precision == DMC_FP64)
    hipLaunchKernelGGL((k_oi_batch<TMAX, 32, KR, double>), dim3(njobs), dim3(NT), 0, st, args, jobs);
  else
    hipLaunchKernelGGL((k_oi_batch<TMAX, 32, KR, float>), dim3(njobs), dim3(NT), 0, st, args, jobs);
}

}  // namespace dmc
