// Supernodal triangular solves with the Cholesky factor of the normal matrix
// (the decoder's preconditioner): z = (L L^T)^{-1} r for every column at once.
//
// Each supernode s (columns a..a+w-1, rows R_s of size m) carries the solve
// operator B_s = [inv(L_ss); L_os inv(L_ss)] (m x w), precomputed on the host.
// Level scheduling over the supernodal tree (supernodes of one level are
// independent):
//   forward, level 0 upwards
//     gather : W_s = r[perm rows of s] - sum of the update rows aimed at s
//     gemm   : [Y_s; U_s] = B_s W_s   (Y_s = solution rows, U_s = update rows
//              for the ancestors, one slot per row of s below its diagonal block)
//   backward, top level downwards
//     gemm   : X_s = B_s^T [Y_s; -X_(R_s below the diagonal block)],
//              z[perm rows of s] = X_s
// Work items are (supernode, 64-row tile) x 64-column tiles: each wave owns 16
// consecutive rows of one 64-column slice and keeps them in registers, so each
// vector load of W, Y or X feeds 16 FMAs and the operator entries are
// wave-uniform scalar loads.
#include "dmc_internal.h"

namespace dmc {
namespace {

constexpr int CT = 64;   // columns per block (one per lane)
constexpr int RT = 64;   // rows per block
constexpr int RPW = 16;  // rows per wave

__global__ void __launch_bounds__(kBlock)
k_fwd_gather(CholDev f, int t0, int ncols, const double* __restrict__ rhs,
             const double* __restrict__ U, double* __restrict__ W) {
  const int task = t0 + blockIdx.x;
  const int s = f.task_w_sn[task], r0 = f.task_w_r0[task];
  const int c = blockIdx.y * CT + threadIdx.x % CT;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
  if (c >= ncols) return;
  const int a = f.sn_start[s], w = f.sn_start[s + 1] - a;
  for (int k = 0; k < RPW; ++k) {
    const int t = r0 + wv * RPW + k;
    if (t >= w) break;
    const int j = a + t;
    double acc = rhs[(size_t)f.perm[j] * ncols + c];
    const int e1 = f.contrib_ptr[j + 1];
    for (int e = f.contrib_ptr[j]; e < e1; ++e) acc -= U[(size_t)f.contrib_slot[e] * ncols + c];
    W[(size_t)j * ncols + c] = acc;
  }
}

__global__ void __launch_bounds__(kBlock)
k_fwd_gemm(CholDev f, int t0, int ncols, const double* __restrict__ W, double* __restrict__ Y,
           double* __restrict__ U) {
  const int task = t0 + blockIdx.x;
  const int s = f.task_m_sn[task], r0 = f.task_m_r0[task];
  const int c = blockIdx.y * CT + threadIdx.x % CT;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
  if (c >= ncols) return;
  const int a = f.sn_start[s], w = f.sn_start[s + 1] - a;
  const int m = f.sn_rowptr[s + 1] - f.sn_rowptr[s];
  const int i0 = r0 + wv * RPW;
  if (i0 >= m) return;
  const double* Bc = f.bcol + f.sn_valptr[s];
  double acc[RPW];
#pragma unroll
  for (int k = 0; k < RPW; ++k) acc[k] = 0.0;
  const double* Wc = W + (size_t)a * ncols + c;
  // rows inside the diagonal block use only the lower triangle of inv(L_ss)
  const int qend = i0 + RPW <= w ? i0 + RPW : w;
  if (i0 + RPW <= m) {
    for (int q = 0; q < qend; ++q) {
      const double x = Wc[(size_t)q * ncols];
      const double* bq = Bc + (size_t)q * m + i0;
#pragma unroll
      for (int k = 0; k < RPW; ++k) acc[k] = fma(bq[k], x, acc[k]);
    }
  } else {
    for (int q = 0; q < qend; ++q) {
      const double x = Wc[(size_t)q * ncols];
      const double* bq = Bc + (size_t)q * m + i0;
#pragma unroll
      for (int k = 0; k < RPW; ++k)
        if (i0 + k < m) acc[k] = fma(bq[k], x, acc[k]);
    }
  }
  const int64_t sb = f.slot_base[s];
#pragma unroll
  for (int k = 0; k < RPW; ++k) {
    const int i = i0 + k;
    if (i >= m) break;
    if (i < w)
      Y[(size_t)(a + i) * ncols + c] = acc[k];
    else
      U[(size_t)(sb + i - w) * ncols + c] = acc[k];
  }
}

__global__ void __launch_bounds__(kBlock)
k_bwd_gemm(CholDev f, int t0, int ncols, const double* __restrict__ Y, double* __restrict__ X,
           double* __restrict__ z) {
  const int task = t0 + blockIdx.x;
  const int s = f.task_w_sn[task], r0 = f.task_w_r0[task];
  const int c = blockIdx.y * CT + threadIdx.x % CT;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
  if (c >= ncols) return;
  const int a = f.sn_start[s], w = f.sn_start[s + 1] - a;
  const int rb = f.sn_rowptr[s], m = f.sn_rowptr[s + 1] - rb;
  const int t0w = r0 + wv * RPW;
  if (t0w >= w) return;
  const double* Br = f.brow + f.sn_valptr[s];
  double acc[RPW];
#pragma unroll
  for (int k = 0; k < RPW; ++k) acc[k] = 0.0;
  const bool full = t0w + RPW <= w;
  // rows of B_s^T: inverse part (i < w; zero for i < t) then the update part
  for (int i = t0w; i < m; ++i) {
    const double v = i < w ? Y[(size_t)(a + i) * ncols + c]
                           : -X[(size_t)f.rowidx[rb + i] * ncols + c];
    const double* bi = Br + (size_t)i * w + t0w;
    if (full) {
#pragma unroll
      for (int k = 0; k < RPW; ++k) acc[k] = fma(bi[k], v, acc[k]);
    } else {
#pragma unroll
      for (int k = 0; k < RPW; ++k)
        if (t0w + k < w) acc[k] = fma(bi[k], v, acc[k]);
    }
  }
#pragma unroll
  for (int k = 0; k < RPW; ++k) {
    const int t = t0w + k;
    if (t >= w) break;
    X[(size_t)(a + t) * ncols + c] = acc[k];
    z[(size_t)f.perm[a + t] * ncols + c] = acc[k];
  }
}

}  // namespace

void launch_chol_solve(hipStream_t s, const CholDev& f, int32_t ncols, const double* r, double* z,
                       double* W, double* Y, double* X, double* U) {
  dim3 blk(kBlock);
  const int cb = (ncols + CT - 1) / CT;
  for (int lv = 0; lv < f.nlevels; ++lv) {
    const int tw0 = f.level_w_host[lv], ntw = f.level_w_host[lv + 1] - tw0;
    const int tm0 = f.level_m_host[lv], ntm = f.level_m_host[lv + 1] - tm0;
    prof::begin(s, DMC_KERNEL_CHOL_FWD_GATHER);
    hipLaunchKernelGGL(k_fwd_gather, dim3(ntw, cb), blk, 0, s, f, tw0, ncols, r, U, W);
    prof::end(s, DMC_KERNEL_CHOL_FWD_GATHER);
    prof::begin(s, DMC_KERNEL_CHOL_FWD_SOLVE);
    hipLaunchKernelGGL(k_fwd_gemm, dim3(ntm, cb), blk, 0, s, f, tm0, ncols, W, Y, U);
    prof::end(s, DMC_KERNEL_CHOL_FWD_SOLVE);
  }
  for (int lv = f.nlevels - 1; lv >= 0; --lv) {
    const int tw0 = f.level_w_host[lv], ntw = f.level_w_host[lv + 1] - tw0;
    prof::begin(s, DMC_KERNEL_CHOL_BWD_SOLVE);
    hipLaunchKernelGGL(k_bwd_gemm, dim3(ntw, cb), blk, 0, s, f, tw0, ncols, Y, X, z);
    prof::end(s, DMC_KERNEL_CHOL_BWD_SOLVE);
  }
}

}  // namespace dmc
