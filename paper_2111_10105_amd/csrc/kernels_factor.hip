// Numeric supernodal Cholesky factorisation of the normal matrix
// L^T L + I_N^T I_N of the anchored system (Eq. 12) on the device, from the
// host's ordering and symbolic analysis, and the solve operators the decoder's
// triangular solves read.
//
// Supernode s owns columns a..a+w-1 and rows R_s (m of them: its own columns,
// then the rows below, ascending); its block L_s (m x w) is row-major at
// sn_valptr[s].  Level by level (the supernodes of a level depend only on
// lower levels):
//   scatter   : L_s = the lower triangle of P M P^T (once, all levels)
//   update    : L_s -= L_d(rows of d in R_s) L_d(rows of d in s's columns)^T
//               for every descendant d with rows in s's columns (left-looking)
//   factor    : L_ss = chol(L_ss), L_os = L_os L_ss^-T (64-column panels)
//   operators : B_s = [I; L_os] L_ss^-1 = [inv(L_ss); L_os inv(L_ss)]
//               (after all levels, by 64-row blocks)
// The update kernel gives one workgroup each 64 x 64 tile of a target block
// and walks the target's descendant segments in a fixed order, so every entry
// is written by one workgroup in one order (deterministic, no atomics).
#include "dmc_internal.h"

namespace dmc {
namespace {

constexpr int FT = 64;   // update tile (target rows x target columns)
constexpr int FKC = 32;  // K slice of the update through LDS

// first index in [lo, hi) with v[index] >= x (v ascending)
__device__ inline int lower_idx(const int32_t* v, int lo, int hi, int32_t x) {
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (v[mid] < x)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// column j's entries of the lower triangle of P M P^T into its supernode's block
__global__ void __launch_bounds__(kBlock) k_fac_scatter(FactorDev f) {
  const int j = blockIdx.x * kBlock + threadIdx.x;
  if (j >= f.n) return;
  const int s = f.sn_of[j];
  const int a = f.sn_start[s], w = f.sn_start[s + 1] - a;
  const int r0 = f.sn_rowptr[s], m = f.sn_rowptr[s + 1] - r0;
  const int32_t* R = f.rowidx + r0;
  double* Ls = f.L + f.sn_valptr[s];
  for (int e = f.acol_ptr[j]; e < f.acol_ptr[j + 1]; ++e) {
    const int t = lower_idx(R, 0, m, f.acol_row[e]);
    Ls[(size_t)t * w + (j - a)] = f.acol_val[e];
  }
}

// One 64 x 64 tile (rows tr0.., columns tc0.. of target s) minus every
// descendant's contribution.  For segment (d, p1, p2): the columns are d's
// rows qi in [p1, p2) whose indices fall in the tile's columns, the rows are
// d's rows ri >= qi whose indices fall in the tile's rows (both ranges by
// binary search: d's rows below p1 are rows of s, in the same order); the
// product L_d[ri] . L_d[qi] over d's w_d columns goes through LDS in 32-deep
// slices, thread (y, x) holding a 4 x 4 block of it.
__global__ void __launch_bounds__(kBlock)
k_fac_update(FactorDev f, const int32_t* __restrict__ tile_sn, const int32_t* __restrict__ tile_rc,
             int t0) {
  __shared__ double As[FT][FKC + 1];
  __shared__ double Bs[FT][FKC + 1];
  __shared__ int rowloc[FT], colloc[FT];
  const int task = t0 + blockIdx.x;
  const int s = tile_sn[task], rc = tile_rc[task];
  const int a = f.sn_start[s], w = f.sn_start[s + 1] - a;
  const int rs0 = f.sn_rowptr[s], m = f.sn_rowptr[s + 1] - rs0;
  const int32_t* R = f.rowidx + rs0;
  const int tr0 = (rc >> 16) * FT, tr1 = min(m, tr0 + FT);
  const int tc0 = (rc & 0xffff) * FT, tc1 = min(w, tc0 + FT);
  double* Ls = f.L + f.sn_valptr[s];
  const int tid = threadIdx.x, ty = tid / 16, tx = tid % 16;
  for (int g = f.seg_ptr[s]; g < f.seg_ptr[s + 1]; ++g) {
    const int d = f.seg_d[g], p1 = f.seg_p1[g], p2 = f.seg_p2[g];
    const int rd0 = f.sn_rowptr[d], md = f.sn_rowptr[d + 1] - rd0;
    const int wd = f.sn_start[d + 1] - f.sn_start[d];
    const int32_t* Rd = f.rowidx + rd0;
    const int q_lo = lower_idx(Rd, p1, p2, a + tc0), q_hi = lower_idx(Rd, q_lo, p2, a + tc1);
    if (q_lo >= q_hi) continue;
    const int r_lo = lower_idx(Rd, q_lo, md, R[tr0]), r_hi = lower_idx(Rd, r_lo, md, R[tr1 - 1] + 1);
    if (r_lo >= r_hi) continue;
    const int nr = r_hi - r_lo, nq = q_hi - q_lo;  // both <= 64 (distinct rows / columns of the tile)
    __syncthreads();  // the previous segment's LDS reads are done
    if (tid < nr) rowloc[tid] = lower_idx(R, tr0, tr1, Rd[r_lo + tid]);
    if (tid >= 64 && tid - 64 < nq) colloc[tid - 64] = Rd[q_lo + tid - 64] - a;
    const double* Ld = f.L + f.sn_valptr[d];
    double acc[4][4] = {};
    for (int k0 = 0; k0 < wd; k0 += FKC) {
      __syncthreads();
      for (int e = tid; e < FT * FKC; e += kBlock) {
        const int r = e / FKC, k = e % FKC;
        const bool kv = k0 + k < wd;
        As[r][k] = (r < nr && kv) ? Ld[(size_t)(r_lo + r) * wd + k0 + k] : 0.0;
        Bs[r][k] = (r < nq && kv) ? Ld[(size_t)(q_lo + r) * wd + k0 + k] : 0.0;
      }
      __syncthreads();
#pragma unroll 4
      for (int k = 0; k < FKC; ++k) {
        double av[4], bv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          av[u] = As[ty * 4 + u][k];
          bv[u] = Bs[tx * 4 + u][k];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[u][v] = fma(av[u], bv[v], acc[u][v]);
      }
    }
    // subtract the lower trapezoid (row index >= column index in d)
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int r = ty * 4 + u;
      if (r >= nr) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int q = tx * 4 + v;
        if (q >= nq || r_lo + r < q_lo + q) continue;
        Ls[(size_t)rowloc[r] * w + colloc[q]] -= acc[u][v];
      }
    }
  }
}

// Blocked Cholesky of the level's supernodes, 64-column panel p at a time
// (three launches per panel, all supernodes of the level together):
//   diag  : D = L[P][P] (the panel's diagonal block) factorised in LDS
//   trsm  : L[R][P] = L[R][P] D^-T for every 64-row block R below it
//   update: L[R][Q] -= L[R][P] L[Q][P]^T for the trailing column blocks Q of
//           the supernode's own columns and every row block R >= Q
// Only the lower triangles of the diagonal blocks are ever read.  A
// non-positive pivot marks the supernode in *fail (smallest index + 1).
constexpr int FP = 64;  // panel width

__global__ void __launch_bounds__(kBlock)
k_fac_diag(FactorDev f, const int32_t* __restrict__ lv_sn, int s0, int p) {
  __shared__ double D[FP][FP + 1];
  __shared__ int bad;
  const int s = lv_sn[s0 + blockIdx.x];
  const int w = f.sn_start[s + 1] - f.sn_start[s];
  const int c0 = p * FP;
  if (c0 >= w) return;
  const int pw = min(FP, w - c0), tid = threadIdx.x;
  double* Ls = f.L + f.sn_valptr[s];
  for (int e = tid; e < pw * pw; e += kBlock) {
    const int r = e / pw, c = e % pw;
    if (c <= r) D[r][c] = Ls[(size_t)(c0 + r) * w + c0 + c];
  }
  if (tid == 0) bad = 0;
  __syncthreads();
  for (int j = 0; j < pw; ++j) {
    if (tid == 0) {
      double d = D[j][j];
      if (!(d > 0.0)) {
        bad = 1;
        d = 1.0;
      }
      D[j][j] = sqrt(d);
    }
    __syncthreads();
    for (int i = j + 1 + tid; i < pw; i += kBlock) D[i][j] /= D[j][j];
    __syncthreads();
    // trailing lower triangle: entries (i, k) with j < k <= i < pw
    const int t = pw - 1 - j;  // trailing size
    for (int e = tid; e < t * t; e += kBlock) {
      const int i = j + 1 + e / t, k = j + 1 + e % t;
      if (k <= i) D[i][k] -= D[i][j] * D[k][j];
    }
    __syncthreads();
  }
  for (int e = tid; e < pw * pw; e += kBlock) {
    const int r = e / pw, c = e % pw;
    if (c <= r) Ls[(size_t)(c0 + r) * w + c0 + c] = D[r][c];
  }
  if (tid == 0 && bad) atomicMin(f.fail, s + 1);
}

// block (supernode, row block rb >= p): the block's rows below the panel's
// diagonal block (rows from c0 + pw on; in row block p only when the panel
// is the supernode's last and narrower than 64) solved against it,
// x_j = (x_j - sum_{k<j} x_k D[j][k]) / D[j][j] (thread r owns row r)
__global__ void __launch_bounds__(kBlock)
k_fac_trsm(FactorDev f, const int32_t* __restrict__ lv_sn, int s0, int p) {
  __shared__ double D[FP][FP + 1];
  __shared__ double X[FP][FP + 1];
  const int s = lv_sn[s0 + blockIdx.x], rb = blockIdx.y;
  const int w = f.sn_start[s + 1] - f.sn_start[s];
  const int m = f.sn_rowptr[s + 1] - f.sn_rowptr[s];
  const int c0 = p * FP;
  if (c0 >= w || rb < p) return;
  const int pw = min(FP, w - c0), tid = threadIdx.x;
  const int r0 = max(rb * FP, c0 + pw), nr = min(rb * FP + FP, m) - r0;
  if (nr <= 0) return;
  double* Ls = f.L + f.sn_valptr[s];
  for (int e = tid; e < FP * FP; e += kBlock) {
    const int r = e / FP, c = e % FP;
    if (r < pw && c <= r) D[r][c] = Ls[(size_t)(c0 + r) * w + c0 + c];
    if (r < nr && c < pw) X[r][c] = Ls[(size_t)(r0 + r) * w + c0 + c];
  }
  __syncthreads();
  if (tid < nr) {
    for (int j = 0; j < pw; ++j) {
      double x = X[tid][j];
      for (int k = 0; k < j; ++k) x -= X[tid][k] * D[j][k];
      X[tid][j] = x / D[j][j];
    }
  }
  __syncthreads();
  for (int e = tid; e < nr * pw; e += kBlock) {
    const int r = e / pw, c = e % pw;
    Ls[(size_t)(r0 + r) * w + c0 + c] = X[r][c];
  }
}

// block (supernode, row block rb, column block cb > p with rb >= cb):
// L[rb][cb] -= L[rb][p] L[cb][p]^T (64 x 64 x 64 through LDS in 32-deep
// slices, thread (y, x) holding a 4 x 4 block)
__global__ void __launch_bounds__(kBlock)
k_fac_trail(FactorDev f, const int32_t* __restrict__ lv_sn, int s0, int p) {
  __shared__ double As[FT][FKC + 1];
  __shared__ double Bs[FT][FKC + 1];
  const int s = lv_sn[s0 + blockIdx.x], rb = blockIdx.y, cb = blockIdx.z;
  const int w = f.sn_start[s + 1] - f.sn_start[s];
  const int m = f.sn_rowptr[s + 1] - f.sn_rowptr[s];
  const int c0 = p * FP, q0 = cb * FP, r0 = rb * FP;
  if (cb <= p || q0 >= w || rb < cb || r0 >= m) return;
  const int pw = min(FP, w - c0), nq = min(FP, w - q0), nr = min(FP, m - r0);
  const int tid = threadIdx.x, ty = tid / 16, tx = tid % 16;
  double* Ls = f.L + f.sn_valptr[s];
  double acc[4][4] = {};
  for (int k0 = 0; k0 < pw; k0 += FKC) {
    __syncthreads();
    for (int e = tid; e < FT * FKC; e += kBlock) {
      const int r = e / FKC, k = e % FKC;
      const bool kv = k0 + k < pw;
      As[r][k] = (r < nr && kv) ? Ls[(size_t)(r0 + r) * w + c0 + k0 + k] : 0.0;
      Bs[r][k] = (r < nq && kv) ? Ls[(size_t)(q0 + r) * w + c0 + k0 + k] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int k = 0; k < FKC; ++k) {
      double av[4], bv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        av[u] = As[ty * 4 + u][k];
        bv[u] = Bs[tx * 4 + u][k];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = fma(av[u], bv[v], acc[u][v]);
    }
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int r = ty * 4 + u;
    if (r >= nr) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int q = tx * 4 + v;
      if (q >= nq) continue;
      Ls[(size_t)(r0 + r) * w + q0 + q] -= acc[u][v];
    }
  }
}

// B_s = [I; L_os] L_ss^-1 by 64-row blocks (block = supernode, row block):
// panels from the last to the first, B[rows][P] = (C[rows][P] - B[rows][>P]
// L[>P][P]) L[P][P]^-1 with C the identity on the diagonal block's rows and
// L_os below it; the product through LDS as in k_fac_trail, the triangular
// part by rows (b_j = (x_j - sum_{k>j} b_k D[k][j]) / D[j][j]).  The rows of
// the diagonal block come out lower triangular (exact zeros above).
__global__ void __launch_bounds__(kBlock)
k_fac_operators(FactorDev f, const int32_t* __restrict__ op_sn, const int32_t* __restrict__ op_row,
                int t0) {
  __shared__ double As[FT][FKC + 1];
  __shared__ double Bs[FT][FKC + 1];
  __shared__ double D[FP][FP + 1];
  __shared__ double X[FP][FP + 1];
  const int task = t0 + blockIdx.x;
  const int s = op_sn[task], r0 = op_row[task];
  const int w = f.sn_start[s + 1] - f.sn_start[s];
  const int m = f.sn_rowptr[s + 1] - f.sn_rowptr[s];
  const int nr = min(FP, m - r0);
  const int tid = threadIdx.x, ty = tid / 16, tx = tid % 16;
  const double* Ls = f.L + f.sn_valptr[s];
  double* Bm = f.B + f.sn_valptr[s];
  const int npan = (w + FP - 1) / FP;
  for (int P = npan - 1; P >= 0; --P) {
    const int c0 = P * FP, pw = min(FP, w - c0);
    double acc[4][4] = {};
    // B[rows][k] L[k][c0 + c] over the later columns k >= c0 + pw
    for (int k0 = c0 + pw; k0 < w; k0 += FKC) {
      __syncthreads();
      for (int e = tid; e < FT * FKC; e += kBlock) {
        const int r = e / FKC, k = e % FKC;
        const bool kv = k0 + k < w;
        As[r][k] = (r < nr && kv) ? Bm[(size_t)(r0 + r) * w + k0 + k] : 0.0;
        // Bs[c][k] = L[k0 + k][c0 + c]
        Bs[r][k] = (r < pw && kv) ? Ls[(size_t)(k0 + k) * w + c0 + r] : 0.0;
      }
      __syncthreads();
#pragma unroll 4
      for (int k = 0; k < FKC; ++k) {
        double av[4], bv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          av[u] = As[ty * 4 + u][k];
          bv[u] = Bs[tx * 4 + u][k];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[u][v] = fma(av[u], bv[v], acc[u][v]);
      }
    }
    __syncthreads();
    for (int e = tid; e < FP * FP; e += kBlock) {
      const int r = e / FP, c = e % FP;
      if (r < pw && c <= r) D[r][c] = Ls[(size_t)(c0 + r) * w + c0 + c];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int r = ty * 4 + u, i = r0 + r;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int c = tx * 4 + v;
        if (r >= nr || c >= pw) continue;
        const double cv = i < w ? (i == c0 + c ? 1.0 : 0.0) : Ls[(size_t)i * w + c0 + c];
        X[r][c] = cv - acc[u][v];
      }
    }
    __syncthreads();
    if (tid < nr) {
      for (int j = pw - 1; j >= 0; --j) {
        double x = X[tid][j];
        for (int k = j + 1; k < pw; ++k) x -= X[tid][k] * D[k][j];
        X[tid][j] = x / D[j][j];
      }
    }
    __syncthreads();
    for (int e = tid; e < nr * pw; e += kBlock) {
      const int r = e / pw, c = e % pw;
      Bm[(size_t)(r0 + r) * w + c0 + c] = X[r][c];
    }
  }
}

// out[r] = in[map[r]], rows of ncols doubles
__global__ void __launch_bounds__(kBlock)
k_permute_rows(const double* __restrict__ in, const int32_t* __restrict__ map, int n, int ncols,
               double* __restrict__ out) {
  const size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= (size_t)n * ncols) return;
  const size_t r = e / ncols, c = e % ncols;
  out[e] = in[(size_t)map[r] * ncols + c];
}

}  // namespace

void launch_factor_numeric(hipStream_t s, const FactorDev& f, const FactorPlan& p) {
  hipLaunchKernelGGL(k_fac_scatter, dim3((f.n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, f);
  for (int lv = 0; lv < p.nlevels; ++lv) {
    const int nt = p.tile_off[lv + 1] - p.tile_off[lv];
    if (nt > 0)
      hipLaunchKernelGGL(k_fac_update, dim3(nt), dim3(kBlock), 0, s, f, p.tile_sn, p.tile_rc,
                         p.tile_off[lv]);
    const int ns = p.sn_off[lv + 1] - p.sn_off[lv], s0 = p.sn_off[lv];
    const int nrb = (p.maxm[lv] + FP - 1) / FP, npan = (p.maxw[lv] + FP - 1) / FP;
    for (int q = 0; q < npan; ++q) {
      hipLaunchKernelGGL(k_fac_diag, dim3(ns), dim3(kBlock), 0, s, f, p.lv_sn, s0, q);
      hipLaunchKernelGGL(k_fac_trsm, dim3(ns, nrb), dim3(kBlock), 0, s, f, p.lv_sn, s0, q);
      if (npan > q + 1)
        hipLaunchKernelGGL(k_fac_trail, dim3(ns, nrb, npan), dim3(kBlock), 0, s, f, p.lv_sn, s0,
                           q);
    }
  }
  if (p.op_off_total > 0)
    hipLaunchKernelGGL(k_fac_operators, dim3(p.op_off_total), dim3(kBlock), 0, s, f, p.op_sn,
                       p.op_row, 0);
}

void launch_permute_rows(hipStream_t s, const double* in, const int32_t* map, int32_t n,
                         int32_t ncols, double* out) {
  const size_t tot = (size_t)n * ncols;
  if (tot == 0) return;
  hipLaunchKernelGGL(k_permute_rows, dim3((tot + kBlock - 1) / kBlock), dim3(kBlock), 0, s, in, map,
                     n, ncols, out);
}

}  // namespace dmc
