// Lane moves and whole-wavefront reductions of doubles on CDNA (64 lanes),
// shared by the kernels of the library.
#pragma once
#include <hip/hip_runtime.h>

namespace dmc {

// DPP lane moves of a double (both halves): DPP_ROW_MIRROR (0x140) gives lane t
// of each 16-lane row the value of lane 15 - t; DPP_WAVE_ROR1 (0x13C) gives
// lane t the value of lane t - 1 (mod 64).
constexpr int kDppRowMirror = 0x140, kDppWaveRor1 = 0x13C;

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffLL), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ double shfl_f64(double v, int src) {
  const long long b = __double_as_longlong(v);
  const int lo = __shfl((int)(b & 0xffffffffLL), src);
  const int hi = __shfl((int)(b >> 32), src);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Value of v held by lane (l ^ 16) for lane l (swizzle within 32 lanes).
__device__ __forceinline__ double swap16_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_ds_swizzle((int)(b & 0xffffffffLL), 0x401F);
  const int hi = __builtin_amdgcn_ds_swizzle((int)(b >> 32), 0x401F);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sums / maxima over the wavefront (the whole workgroup), the same value in
// every lane: within each 16-lane row by DPP (quad_perm [1,0,3,2] and
// [2,3,0,1], row_half_mirror, row_mirror: each step pairs a lane with one
// holding the other half of its group), the two rows of each 32-lane half by
// a swizzle, the halves by lane reads.  Each step adds a value and its
// partner's in the same order on both lanes, so every lane gets the same bits.
template <typename Op>
__device__ __forceinline__ double wave_reduce(double v, Op op) {
  v = op(v, dpp_f64<0xB1>(v));
  v = op(v, dpp_f64<0x4E>(v));
  v = op(v, dpp_f64<0x141>(v));
  v = op(v, dpp_f64<kDppRowMirror>(v));
  v = op(v, swap16_f64(v));
  return op(readlane_f64(v, 0), readlane_f64(v, 32));
}

__device__ __forceinline__ double wave_sum(double v) {
  return wave_reduce(v, [](double a, double b) { return a + b; });
}

// N independent sums over the wavefront, stage by stage (the N lane moves of
// a stage are issued together, and the N swizzles share one wait); each sum
// takes the same steps in the same order as wave_sum, so it has its bits.
template <int N>
__device__ __forceinline__ void wave_sum_n(double (&v)[N]) {
  double t[N];
#pragma unroll
  for (int i = 0; i < N; ++i) t[i] = dpp_f64<0xB1>(v[i]);
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] += t[i];
#pragma unroll
  for (int i = 0; i < N; ++i) t[i] = dpp_f64<0x4E>(v[i]);
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] += t[i];
#pragma unroll
  for (int i = 0; i < N; ++i) t[i] = dpp_f64<0x141>(v[i]);
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] += t[i];
#pragma unroll
  for (int i = 0; i < N; ++i) t[i] = dpp_f64<kDppRowMirror>(v[i]);
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] += t[i];
#pragma unroll
  for (int i = 0; i < N; ++i) t[i] = swap16_f64(v[i]);
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] += t[i];
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] = readlane_f64(v[i], 0) + readlane_f64(v[i], 32);
}
__device__ __forceinline__ double wave_min(double v) {
  return wave_reduce(v, [](double a, double b) { return fmin(a, b); });
}
__device__ __forceinline__ double wave_max(double v) {
  return wave_reduce(v, [](double a, double b) { return fmax(a, b); });
}

}  // namespace dmc
