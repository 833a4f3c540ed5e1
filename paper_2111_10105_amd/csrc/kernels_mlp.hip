// Learned start of the orthogonal iterations: a row-wise three-layer
// perceptron on the sketch of each window's autocorrelation (Eq. 7).
//
//   sketch   S = R Omega (T x 32), columns orthonormalised, times sqrt(T)
//            (float64)
//   forward  h1 = gelu(S W1 + b1), h2 = gelu(h1 W2 + b2), Q = h2 W3 + b3
//            bfloat16 operands on the matrix cores
//            (v_mfma_f32_16x16x32_bf16), float32 accumulation
//   loss     per (window, coordinate) block: ||(I - U U^T) Q||^2 / ||Q||^2
//            + mu ||Q^T Q / (||Q||^2 / k) - I||^2, and dl/dQ
//   backward float32 with the bfloat16-rounded weights; per-workgroup
//            partial gradients summed in a fixed order (deterministic)
//   adam     bias-corrected Adam on the float32 master weights
//
// Parameters are one float32 vector: W1 [32][128], b1 [128], W2 [128][128],
// b2 [128], W3 [128][k], b3 [k], row-major, in this order.
#include "dmc_internal.h"

namespace dmc {
namespace {

constexpr int SK = 32;   // sketch columns
constexpr int HD = 128;  // hidden width
constexpr int KO = 32;   // output columns, padded

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float gelu(float x) { return x * 0.5f * erfcf(-x * 0.70710678118654752f); }
__device__ __forceinline__ float gelu_grad(float x) {
  return 0.5f * erfcf(-x * 0.70710678118654752f) + x * 0.39894228040143268f * __expf(-0.5f * x * x);
}
__device__ __forceinline__ float bf16r(float x) { return (float)(__bf16)x; }

struct MlpOffsets {
  int w1, b1, w2, b2, w3, b3, count;
};
__host__ __device__ inline MlpOffsets mlp_offsets(int k) {
  MlpOffsets o;
  o.w1 = 0;
  o.b1 = o.w1 + SK * HD;
  o.w2 = o.b1 + HD;
  o.b2 = o.w2 + HD * HD;
  o.w3 = o.b2 + HD;
  o.b3 = o.w3 + HD * k;
  o.count = o.b3 + k;
  return o;
}

// ---- sketch features: one workgroup (one wavefront) per block, lane = row --
// S = R Omega in float64, its columns orthonormalised by classical
// Gram-Schmidt run twice per column (column order), a column keeping less
// than kDrop of its norm after the projections set to zero, then scaled by
// sqrt(T).  The columns of R Omega differ in size by the eigenvalue spread of
// the uncentred R; orthonormalising exposes the smaller directions.
constexpr double kDrop = 1e-10;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

__global__ void __launch_bounds__(64) k_mlp_sketch(const double* __restrict__ R, int T,
                                                   const double* __restrict__ omega,
                                                   float* __restrict__ S) {
  const int b = blockIdx.x, t = threadIdx.x;
  const double* Rb = R + (size_t)b * T * T;
  double a[SK];
#pragma unroll
  for (int j = 0; j < SK; ++j) a[j] = 0.0;
  if (t < T) {
    for (int i = 0; i < T; ++i) {
      const double r = Rb[(size_t)t * T + i];
#pragma unroll
      for (int j = 0; j < SK; ++j) a[j] = fma(r, omega[i * SK + j], a[j]);
    }
  }
  // columns 0..j-1 of a hold the finished (orthonormal or zero) columns
#pragma unroll
  for (int j = 0; j < SK; ++j) {
    double v = a[j];
    const double n0 = sqrt(wave_sum(v * v));
#pragma unroll
    for (int pass = 0; pass < 2; ++pass) {
      double d[SK];
#pragma unroll
      for (int l = 0; l < j; ++l) d[l] = wave_sum(a[l] * v);
#pragma unroll
      for (int l = 0; l < j; ++l) v = fma(-d[l], a[l], v);
    }
    const double nj = sqrt(wave_sum(v * v));
    a[j] = (n0 > 0.0 && nj > kDrop * n0) ? v / nj : 0.0;
  }
  if (t < T) {
    const double sc = sqrt((double)T);
    float* Sb = S + ((size_t)b * T + t) * SK;
#pragma unroll
    for (int j = 0; j < SK; ++j) Sb[j] = (float)(a[j] * sc);
  }
}

// ---- forward: 64 rows per workgroup, 4 waves of 16 rows ------------------
constexpr int FR = 64;          // rows per workgroup
constexpr int LS = SK + 8;      // bf16 row strides (16-byte aligned rows)
constexpr int LH = HD + 8;

struct FwdSmem {
  __bf16 S[FR * LS];
  __bf16 W1t[HD * LS];   // W1 transposed: [out][in]
  __bf16 H1[FR * LH];
  __bf16 W2t[HD * LH];
  __bf16 H2[FR * LH];
  __bf16 W3t[KO * LH];
};

__device__ __forceinline__ bf8 ld8(const __bf16* p) { return *(const bf8*)p; }

__global__ void __launch_bounds__(256) k_mlp_fwd(const float* __restrict__ theta, int k,
                                                 const float* __restrict__ S, int N,
                                                 float* __restrict__ Q, float* __restrict__ cache) {
  __shared__ FwdSmem sm;
  const MlpOffsets o = mlp_offsets(k);
  const int tid = threadIdx.x, lane = tid % 64, w = tid / 64;
  const int r16 = lane % 16, q4 = lane / 16;
  const int row0 = blockIdx.x * FR;
  // stage the weights (transposed, bf16) and the input rows
  for (int e = tid; e < SK * HD; e += 256) {
    const int i = e / HD, n = e % HD;  // W1[i][n]
    sm.W1t[n * LS + i] = (__bf16)theta[o.w1 + e];
  }
  for (int e = tid; e < HD * HD; e += 256) {
    const int i = e / HD, n = e % HD;
    sm.W2t[n * LH + i] = (__bf16)theta[o.w2 + e];
  }
  for (int e = tid; e < KO * HD; e += 256) {
    const int n = e / HD, i = e % HD;  // W3t[n][i] = W3[i][n]
    sm.W3t[n * LH + i] = (__bf16)(n < k ? theta[o.w3 + i * k + n] : 0.0f);
  }
  for (int e = tid; e < FR * SK; e += 256) {
    const int r = e / SK, j = e % SK;
    const int row = row0 + r;
    sm.S[r * LS + j] = (__bf16)(row < N ? S[(size_t)row * SK + j] : 0.0f);
  }
  __syncthreads();
  const int rb = w * 16;  // this wave's rows within the tile
  // layer 1: K = 32, one MFMA per 16 x 16 output tile
#pragma unroll
  for (int ct = 0; ct < HD / 16; ++ct) {
    f4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ld8(&sm.S[(rb + r16) * LS + 8 * q4]),
                                                  ld8(&sm.W1t[(ct * 16 + r16) * LS + 8 * q4]), acc, 0, 0, 0);
    const int col = ct * 16 + r16;
    const float bias = theta[o.b1 + col];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = rb + 4 * q4 + r;
      const float z = acc[r] + bias;
      if (cache && row0 + row < N) cache[(size_t)(row0 + row) * (2 * HD) + col] = z;
      sm.H1[row * LH + col] = (__bf16)gelu(z);
    }
  }
  __syncthreads();
  // layer 2: K = 128
#pragma unroll
  for (int ct = 0; ct < HD / 16; ++ct) {
    f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kk = 0; kk < HD; kk += 32)
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ld8(&sm.H1[(rb + r16) * LH + kk + 8 * q4]),
                                                    ld8(&sm.W2t[(ct * 16 + r16) * LH + kk + 8 * q4]), acc,
                                                    0, 0, 0);
    const int col = ct * 16 + r16;
    const float bias = theta[o.b2 + col];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = rb + 4 * q4 + r;
      const float z = acc[r] + bias;
      if (cache && row0 + row < N) cache[(size_t)(row0 + row) * (2 * HD) + HD + col] = z;
      sm.H2[row * LH + col] = (__bf16)gelu(z);
    }
  }
  __syncthreads();
  // layer 3: K = 128, k <= 32 outputs
#pragma unroll
  for (int ct = 0; ct < KO / 16; ++ct) {
    f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kk = 0; kk < HD; kk += 32)
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ld8(&sm.H2[(rb + r16) * LH + kk + 8 * q4]),
                                                    ld8(&sm.W3t[(ct * 16 + r16) * LH + kk + 8 * q4]), acc,
                                                    0, 0, 0);
    const int col = ct * 16 + r16;
    if (col < k) {
      const float bias = theta[o.b3 + col];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = row0 + rb + 4 * q4 + r;
        if (row < N) Q[(size_t)row * k + col] = acc[r] + bias;
      }
    }
  }
}

// ---- loss and dl/dQ per block (one workgroup per block) -------------------
__global__ void __launch_bounds__(256) k_mlp_loss(const float* __restrict__ Q, const double* __restrict__ U,
                                                  int T, int k, int nb, double mu,
                                                  float* __restrict__ dQ, double* __restrict__ loss) {
  __shared__ float Qs[64 * 33], Us[64 * 33];
  __shared__ float G[32 * 33], A[32 * 33];
  __shared__ double red[3][256];
  const int b = blockIdx.x, tid = threadIdx.x;
  const float* Qb = Q + (size_t)b * T * k;
  const double* Ub = U + (size_t)b * T * k;
  for (int e = tid; e < T * k; e += 256) {
    Qs[(e / k) * 33 + e % k] = Qb[e];
    Us[(e / k) * 33 + e % k] = (float)Ub[e];
  }
  __syncthreads();
  double n2 = 0.0, a2 = 0.0;
  for (int e = tid; e < k * k; e += 256) {
    const int a = e / k, c = e % k;
    float g = 0.f, h = 0.f;
    for (int t = 0; t < T; ++t) {
      g = fmaf(Qs[t * 33 + a], Qs[t * 33 + c], g);
      h = fmaf(Us[t * 33 + a], Qs[t * 33 + c], h);
    }
    G[a * 33 + c] = g;
    A[a * 33 + c] = h;
    if (a == c) n2 += g;
    a2 += (double)h * h;
  }
  red[0][tid] = n2;
  red[1][tid] = a2;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) {
      red[0][tid] += red[0][tid + s];
      red[1][tid] += red[1][tid + s];
    }
    __syncthreads();
  }
  n2 = red[0][0];
  a2 = red[1][0];
  __syncthreads();
  const double c = (double)k / n2;
  double mm = 0.0, mg = 0.0;
  for (int e = tid; e < k * k; e += 256) {
    const int a = e / k, cc = e % k;
    const double m = c * G[a * 33 + cc] - (a == cc ? 1.0 : 0.0);
    mm += m * m;
    mg += m * G[a * 33 + cc];
  }
  red[0][tid] = mm;
  red[1][tid] = mg;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) {
      red[0][tid] += red[0][tid + s];
      red[1][tid] += red[1][tid + s];
    }
    __syncthreads();
  }
  mm = red[0][0];
  mg = red[1][0];
  const double inv_nb = 1.0 / nb;
  const double cq = (2.0 * a2 / (n2 * n2) - mu * 4.0 * k * mg / (n2 * n2)) * inv_nb;
  const double cu = -2.0 / n2 * inv_nb;
  const double cm = mu * 4.0 * c * inv_nb;
  for (int e = tid; e < T * k; e += 256) {
    const int t = e / k, j = e % k;
    float ua = 0.f, qm = 0.f;
    for (int a = 0; a < k; ++a) {
      ua = fmaf(Us[t * 33 + a], A[a * 33 + j], ua);
      const float mij = (float)(c * G[a * 33 + j] - (a == j ? 1.0 : 0.0));
      qm = fmaf(Qs[t * 33 + a], mij, qm);
    }
    dQ[(size_t)b * T * k + e] = (float)(cu * ua + cq * Qs[t * 33 + j] + cm * qm);
  }
  if (tid == 0 && loss) loss[b] = (1.0 - a2 / n2) + mu * mm;
}

// ---- backward ------------------------------------------------------------
// (1) activation gradients per 32-row tile: dZ2 = (dQ W3^T) gelu'(Z2),
//     dZ1 = (dZ2 W2^T) gelu'(Z1), written as dZ [N][256] (dZ1 | dZ2);
// (2) weight gradients dW3 = H2^T dQ, dW2 = H1^T dZ2, dW1 = S^T dZ1 and the
//     bias sums, each workgroup over a contiguous range of tiles, into its own
//     partial vector; (3) the partials summed in a fixed order.
constexpr int BR = 32;
constexpr int LB = HD + 1;

struct ActSmem {
  float dQ[BR * (KO + 1)];
  float Z1[BR * LB];
  float Z2[BR * LB];
  float dZ2[BR * LB];
  __bf16 W2[HD * HD];       // bf16-rounded W2 [in][out]
  float W3[HD * (KO + 1)];  // bf16-rounded W3 [in][out]
};

__global__ void __launch_bounds__(256) k_mlp_bwd_act(const float* __restrict__ theta, int k, int N,
                                                     const float* __restrict__ cache,
                                                     const float* __restrict__ dQg,
                                                     float* __restrict__ dZ) {
  __shared__ ActSmem sm;
  const MlpOffsets o = mlp_offsets(k);
  const int tid = threadIdx.x;
  const int row0 = blockIdx.x * BR;
  for (int e = tid; e < HD * HD; e += 256) sm.W2[e] = (__bf16)theta[o.w2 + e];
  for (int e = tid; e < HD * KO; e += 256) {
    const int i = e / KO, c = e % KO;
    sm.W3[i * (KO + 1) + c] = c < k ? bf16r(theta[o.w3 + i * k + c]) : 0.0f;
  }
  for (int e = tid; e < BR * KO; e += 256) {
    const int r = e / KO, c = e % KO, row = row0 + r;
    sm.dQ[r * (KO + 1) + c] = (row < N && c < k) ? dQg[(size_t)row * k + c] : 0.0f;
  }
  for (int e = tid; e < BR * HD; e += 256) {
    const int r = e / HD, j = e % HD, row = row0 + r;
    sm.Z1[r * LB + j] = row < N ? cache[(size_t)row * 2 * HD + j] : 0.0f;
    sm.Z2[r * LB + j] = row < N ? cache[(size_t)row * 2 * HD + HD + j] : 0.0f;
  }
  __syncthreads();
  // dZ2: thread owns column j and rows rq..rq+15
  {
    const int j = tid % HD, rq = (tid / HD) * 16;
    float w3[KO];
#pragma unroll
    for (int c = 0; c < KO; ++c) w3[c] = sm.W3[j * (KO + 1) + c];
    for (int r = rq; r < rq + 16; ++r) {
      float d = 0.f;
#pragma unroll
      for (int c = 0; c < KO; ++c) d = fmaf(sm.dQ[r * (KO + 1) + c], w3[c], d);
      const float v = d * gelu_grad(sm.Z2[r * LB + j]);
      sm.dZ2[r * LB + j] = v;
      if (row0 + r < N) dZ[(size_t)(row0 + r) * 2 * HD + HD + j] = v;
    }
  }
  __syncthreads();
  // dZ1: thread owns column i and rows rq..rq+15
  {
    const int i = tid % HD, rq = (tid / HD) * 16;
    float acc[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) acc[u] = 0.f;
    for (int j0 = 0; j0 < HD; j0 += 16) {
      float w2[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) w2[u] = (float)sm.W2[i * HD + j0 + u];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        float a = acc[u];
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) a = fmaf(sm.dZ2[(rq + u) * LB + j0 + jj], w2[jj], a);
        acc[u] = a;
      }
    }
    for (int u = 0; u < 16; ++u) {
      const int r = rq + u;
      if (row0 + r < N) dZ[(size_t)(row0 + r) * 2 * HD + i] = acc[u] * gelu_grad(sm.Z1[r * LB + i]);
    }
  }
}

struct WgtSmem {
  float S[BR * (SK + 1)];
  float dQ[BR * (KO + 1)];
  float H1[BR * LB];
  float H2[BR * LB];
  float dZ1[BR * LB];
  float dZ2[BR * LB];
};

__global__ void __launch_bounds__(256) k_mlp_bwd_w(int k, const float* __restrict__ S, int N,
                                                   const float* __restrict__ cache,
                                                   const float* __restrict__ dQg,
                                                   const float* __restrict__ dZ,
                                                   float* __restrict__ partial) {
  __shared__ WgtSmem sm;
  const MlpOffsets o = mlp_offsets(k);
  const int tid = threadIdx.x;
  float gW3[16], gW2[64], gW1[16];
  float gb1 = 0.f, gb2 = 0.f, gb3 = 0.f;
#pragma unroll
  for (int u = 0; u < 16; ++u) gW3[u] = gW1[u] = 0.f;
#pragma unroll
  for (int u = 0; u < 64; ++u) gW2[u] = 0.f;
  const int ntiles = (N + BR - 1) / BR;
  const int per = (ntiles + gridDim.x - 1) / gridDim.x;
  const int t_begin = blockIdx.x * per, t_end = min(ntiles, t_begin + per);
  const int i = tid / 2;                              // rows of dW3, dW2
  const int c0 = (tid % 2) * 16, j0 = (tid % 2) * 64;  // their columns
  const int i1 = tid / 8, j1 = (tid % 8) * 16;        // dW1
  for (int tile = t_begin; tile < t_end; ++tile) {
    const int row0 = tile * BR;
    __syncthreads();
    for (int e = tid; e < BR * SK; e += 256) {
      const int r = e / SK, j = e % SK, row = row0 + r;
      sm.S[r * (SK + 1) + j] = row < N ? S[(size_t)row * SK + j] : 0.0f;
    }
    for (int e = tid; e < BR * KO; e += 256) {
      const int r = e / KO, c = e % KO, row = row0 + r;
      sm.dQ[r * (KO + 1) + c] = (row < N && c < k) ? dQg[(size_t)row * k + c] : 0.0f;
    }
    for (int e = tid; e < BR * HD; e += 256) {
      const int r = e / HD, j = e % HD, row = row0 + r;
      const bool ok = row < N;
      sm.H1[r * LB + j] = ok ? gelu(cache[(size_t)row * 2 * HD + j]) : 0.0f;
      sm.H2[r * LB + j] = ok ? gelu(cache[(size_t)row * 2 * HD + HD + j]) : 0.0f;
      sm.dZ1[r * LB + j] = ok ? dZ[(size_t)row * 2 * HD + j] : 0.0f;
      sm.dZ2[r * LB + j] = ok ? dZ[(size_t)row * 2 * HD + HD + j] : 0.0f;
    }
    __syncthreads();
    for (int r = 0; r < BR; ++r) {
      const float h2 = sm.H2[r * LB + i], h1 = sm.H1[r * LB + i], sv = sm.S[r * (SK + 1) + i1];
#pragma unroll
      for (int u = 0; u < 16; ++u) gW3[u] = fmaf(h2, sm.dQ[r * (KO + 1) + c0 + u], gW3[u]);
#pragma unroll
      for (int u = 0; u < 64; ++u) gW2[u] = fmaf(h1, sm.dZ2[r * LB + j0 + u], gW2[u]);
#pragma unroll
      for (int u = 0; u < 16; ++u) gW1[u] = fmaf(sv, sm.dZ1[r * LB + j1 + u], gW1[u]);
    }
    if (tid < HD) {
      for (int r = 0; r < BR; ++r) {
        gb2 += sm.dZ2[r * LB + tid];
        gb1 += sm.dZ1[r * LB + tid];
      }
    }
    if (tid < KO)
      for (int r = 0; r < BR; ++r) gb3 += sm.dQ[r * (KO + 1) + tid];
  }
  float* P = partial + (size_t)blockIdx.x * o.count;
#pragma unroll
  for (int u = 0; u < 16; ++u)
    if (c0 + u < k) P[o.w3 + i * k + c0 + u] = gW3[u];
#pragma unroll
  for (int u = 0; u < 64; ++u) P[o.w2 + i * HD + j0 + u] = gW2[u];
#pragma unroll
  for (int u = 0; u < 16; ++u) P[o.w1 + i1 * HD + j1 + u] = gW1[u];
  if (tid < HD) {
    P[o.b2 + tid] = gb2;
    P[o.b1 + tid] = gb1;
  }
  if (tid < k) P[o.b3 + tid] = gb3;
}

__global__ void k_mlp_reduce(const float* __restrict__ partial, int nparts, int count,
                             float* __restrict__ grad) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= count) return;
  float s = 0.f;
  for (int q = 0; q < nparts; ++q) s += partial[(size_t)q * count + p];
  grad[p] = s;
}

__global__ void k_mlp_adam(float* __restrict__ theta, const float* __restrict__ grad,
                           float* __restrict__ m, float* __restrict__ v, int count, float lr,
                           float b1, float b2, float eps, float c1, float c2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= count) return;
  const float g = grad[p];
  const float mn = b1 * m[p] + (1.f - b1) * g;
  const float vn = b2 * v[p] + (1.f - b2) * g * g;
  m[p] = mn;
  v[p] = vn;
  theta[p] -= lr * (mn / c1) / (sqrtf(vn / c2) + eps);
}

}  // namespace

int mlp_param_count(int k) { return mlp_offsets(k).count; }

int mlp_bwd_parts() { return 256; }

void launch_mlp_sketch(hipStream_t s, const double* R, int nb, int T, const double* omega, float* S) {
  hipLaunchKernelGGL(k_mlp_sketch, dim3(nb), dim3(64), 0, s, R, T, omega, S);
}

void launch_mlp_forward(hipStream_t s, const float* theta, int k, const float* S, int N, float* Q,
                        float* cache) {
  if (N <= 0) return;
  hipLaunchKernelGGL(k_mlp_fwd, dim3((N + FR - 1) / FR), dim3(256), 0, s, theta, k, S, N, Q, cache);
}

void launch_mlp_loss(hipStream_t s, const float* Q, const double* U, int T, int k, int nb, double mu,
                     float* dQ, double* loss) {
  hipLaunchKernelGGL(k_mlp_loss, dim3(nb), dim3(256), 0, s, Q, U, T, k, nb, mu, dQ, loss);
}

void launch_mlp_backward(hipStream_t s, const float* theta, int k, const float* S, int N,
                         const float* cache, const float* dQ, float* dZ, float* partial,
                         float* grad) {
  const int count = mlp_param_count(k);
  const int parts = mlp_bwd_parts();
  hipLaunchKernelGGL(k_mlp_bwd_act, dim3((N + BR - 1) / BR), dim3(256), 0, s, theta, k, N, cache, dQ,
                     dZ);
  hipLaunchKernelGGL(k_mlp_bwd_w, dim3(parts), dim3(256), 0, s, k, S, N, cache, dQ, dZ, partial);
  hipLaunchKernelGGL(k_mlp_reduce, dim3((count + 255) / 256), dim3(256), 0, s, partial, parts, count,
                     grad);
}

void launch_mlp_adam(hipStream_t s, float* theta, const float* grad, float* m, float* v, int count,
                     int step, double lr, double b1, double b2, double eps) {
  const float c1 = (float)(1.0 - pow(b1, step)), c2 = (float)(1.0 - pow(b2, step));
  hipLaunchKernelGGL(k_mlp_adam, dim3((count + 255) / 256), dim3(256), 0, s, theta, grad, m, v, count,
                     (float)lr, (float)b1, (float)b2, (float)eps, c1, c2);
}

}  // namespace dmc
