// Encoder kernels: delta coordinates (Eq. 3-4, 8), autocorrelation (Eq. 7),
// projection (Eq. 9) with per-row ranges and uniform quantisation (Eq. 10),
// anchor values (Eq. 12).
#include "dmc_internal.h"
#include "wave_ops.h"

namespace dmc {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f16v __attribute__((ext_vector_type(16)));

// ---------------------------------------------------------------------------
// Delta coordinates: one thread per vertex, frames in a loop so the CSR row is
// read once per frame group.  Each ring member's xyz is one 12-byte (float32)
// or 24-byte (float64) load: a wavefront's gather instruction serves three
// coordinates, and the kernel is bound by the number of such instructions
// the texture addressers process, not by HBM bytes.
// uniform:       delta_i = v_i - (1/d_i) sum_{j in ring(i)} v_j    (Eq. 3)
// combinatorial: delta_i = d_i v_i - sum_{j in ring(i)} v_j         (Eq. 1, 4)
// The stencil is evaluated in float64 for both storage types: delta is a small
// difference of nearly equal coordinates, and float32 arithmetic would leave an
// absolute error of the size of one ulp of the coordinates in it.  Each
// coordinate's ring sum is taken in ring order.
// ---------------------------------------------------------------------------
constexpr int DMAX = 8;  // ring members held in registers by k_delta

template <typename Real>
struct Xyz {
  Real x, y, z;
};

template <typename Real>
__global__ void __launch_bounds__(kBlock)
k_delta(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
        const double* __restrict__ w, int uniform, int n, int F, int fpb,
        const Real* __restrict__ in, Real* __restrict__ out) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int e0 = rowptr[i], e1 = rowptr[i + 1];
  const int deg = e1 - e0;
  const double wi = w[i];
  const int t0 = blockIdx.y * fpb;
  const int t1 = min(F, t0 + fpb);
  const size_t fs = (size_t)3 * n;
  // the first DMAX ring members stay in registers, so the loads of a frame
  // are all issued at once (a longer ring reads the rest in a loop)
  int nb[DMAX];
#pragma unroll
  for (int d = 0; d < DMAX; ++d) nb[d] = d < deg ? col[e0 + d] : i;
#pragma unroll 2
  for (int t = t0; t < t1; ++t) {
    const Xyz<Real>* fr = (const Xyz<Real>*)(in + (size_t)t * fs);
    Xyz<Real> v[DMAX];
#pragma unroll
    for (int d = 0; d < DMAX; ++d) v[d] = fr[nb[d]];
    double sx = 0.0, sy = 0.0, sz = 0.0;
#pragma unroll
    for (int d = 0; d < DMAX; ++d)
      if (d < deg) {
        sx += (double)v[d].x;
        sy += (double)v[d].y;
        sz += (double)v[d].z;
      }
    for (int e = e0 + DMAX; e < e1; ++e) {
      const Xyz<Real> u = fr[col[e]];
      sx += (double)u.x;
      sy += (double)u.y;
      sz += (double)u.z;
    }
    const Xyz<Real> own = fr[i];
    Xyz<Real> o;
    o.x = (Real)(uniform ? (double)own.x - wi * sx : wi * (double)own.x - sx);
    o.y = (Real)(uniform ? (double)own.y - wi * sy : wi * (double)own.y - sy);
    o.z = (Real)(uniform ? (double)own.z - wi * sz : wi * (double)own.z - sz);
    ((Xyz<Real>*)(out + (size_t)t * fs))[i] = o;
  }
}

// ---------------------------------------------------------------------------
// Autocorrelation R_c = A_c A_c^T per window (Eq. 7) on the matrix cores.
// Grid (P, nw): block p of window w covers a contiguous vertex range, stages
// tiles of VT vertices x T frames x 3 coordinates in LDS as [c][v][t] (t
// contiguous, padded), and accumulates the upper-triangular output tiles of
// all three coordinates; one wave owns each (coordinate, tile) job.  Partial
// sums go to part[w][p][c][T][T]; a second kernel adds the P partials in a
// fixed order (deterministic) in float64.
// FP32: v_mfma_f32_32x32x2f32 (lane l: A[l%32][l/32], B[l/32][l%32];
//       component r of lane l is D[8(r/4) + 4(l/32) + r%4][l%32]).
// FP64: v_mfma_f64_16x16x4f64 (lane l: A[l%16][l/16], B[l/16][l%16];
//       component r of lane l is D[4r + l/16][l%16]).
// ---------------------------------------------------------------------------
constexpr int AC_VT = 32;      // vertices per LDS tile
constexpr int AC_WAVES = 4;

template <typename Real, int TP>
struct AcTraits;
template <int TP>
struct AcTraits<float, TP> {
  static constexpr int TILE = 32, KSTEP = 2;
  static constexpr int NT = TP / 32;
  static constexpr int JOBS = 3 * NT * (NT + 1) / 2;
  static constexpr int JPW = (JOBS + AC_WAVES - 1) / AC_WAVES;
  typedef f16v acc_t;
  static constexpr int ACC = 16;
};
template <int TP>
struct AcTraits<double, TP> {
  static constexpr int TILE = 16, KSTEP = 4;
  static constexpr int NT = TP / 16;
  static constexpr int JOBS = 3 * NT * (NT + 1) / 2;
  static constexpr int JPW = (JOBS + AC_WAVES - 1) / AC_WAVES;
  typedef d4 acc_t;
  static constexpr int ACC = 4;
};

__device__ inline f16v mfma_step(float a, float b, f16v acc) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
}
__device__ inline d4 mfma_step(double a, double b, d4 acc) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
}

template <typename In, typename Real, int TP>
__global__ void __launch_bounds__(AC_WAVES * 64)
k_autocorr(const In* __restrict__ frames, int n, int T, int nw, int P, Real* __restrict__ part) {
  typedef AcTraits<Real, TP> Tr;
  constexpr int LD = TP + 1;  // padded t stride
  __shared__ Real tile[3 * AC_VT * LD];
  const int p = blockIdx.x, w = blockIdx.y;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int per = (n + P - 1) / P;
  const int v_begin = p * per, v_end = min(n, v_begin + per);
  const In* base = frames + (size_t)w * T * 3 * n;

  typename Tr::acc_t acc[Tr::JPW];
  int jc[Tr::JPW], ji[Tr::JPW], jj[Tr::JPW];
  for (int q = 0; q < Tr::JPW; ++q) {
    for (int r = 0; r < Tr::ACC; ++r) acc[q][r] = 0;
    int job = wave + q * AC_WAVES;
    jc[q] = -1;
    if (job < Tr::JOBS) {
      const int per_c = Tr::NT * (Tr::NT + 1) / 2;
      jc[q] = job / per_c;
      int rem = job % per_c, bi = 0;
      while (rem >= Tr::NT - bi) {
        rem -= Tr::NT - bi;
        ++bi;
      }
      ji[q] = bi;
      jj[q] = bi + rem;
    }
  }
  for (int v0 = v_begin; v0 < v_end; v0 += AC_VT) {
    const int nv = min(AC_VT, v_end - v0);
    __syncthreads();
    // stage: element (t, v, c) of the window -> tile[c][v][t]; zero padding
    for (int e = threadIdx.x; e < TP * 3 * AC_VT; e += AC_WAVES * 64) {
      const int t = e / (3 * AC_VT), rem = e % (3 * AC_VT);
      const int v = rem / 3, c = rem % 3;
      Real val = 0;
      if (t < T && v < nv) val = (Real)base[(size_t)t * 3 * n + (size_t)(v0 + v) * 3 + c];
      tile[(c * AC_VT + v) * LD + t] = val;
    }
    __syncthreads();
    for (int q = 0; q < Tr::JPW; ++q) {
      if (jc[q] < 0) continue;
      const Real* tc = tile + jc[q] * AC_VT * LD;
      const int ra = ji[q] * Tr::TILE + lane % Tr::TILE;
      const int rb = jj[q] * Tr::TILE + lane % Tr::TILE;
      const int kofs = lane / Tr::TILE;
      for (int v = 0; v < AC_VT; v += Tr::KSTEP) {
        const Real a = tc[(v + kofs) * LD + ra];
        const Real b = tc[(v + kofs) * LD + rb];
        acc[q] = mfma_step(a, b, acc[q]);
      }
    }
  }
  // write partial tiles (and the mirrored lower tile)
  Real* out = part + ((size_t)w * P + p) * 3 * TP * TP;
  for (int q = 0; q < Tr::JPW; ++q) {
    if (jc[q] < 0) continue;
    Real* oc = out + (size_t)jc[q] * TP * TP;
    for (int r = 0; r < Tr::ACC; ++r) {
      int row, colx;
      if (Tr::TILE == 32) {
        row = 8 * (r / 4) + 4 * (lane / 32) + (r % 4);
        colx = lane % 32;
      } else {
        row = 4 * r + lane / 16;
        colx = lane % 16;
      }
      const int gi = ji[q] * Tr::TILE + row, gj = jj[q] * Tr::TILE + colx;
      oc[gi * TP + gj] = acc[q][r];
      oc[gj * TP + gi] = acc[q][r];
    }
  }
}

template <typename Real, int TP>
__global__ void k_autocorr_reduce(const Real* __restrict__ part, int T, int nw, int P,
                                  double* __restrict__ R) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int per_w = 3 * T * T;
  if (e >= nw * per_w) return;
  const int w = e / per_w, rem = e % per_w;
  const int c = rem / (T * T), ij = rem % (T * T);
  const int i = ij / T, j = ij % T;
  double s = 0.0;
  for (int p = 0; p < P; ++p)
    s += (double)part[(((size_t)w * P + p) * 3 + c) * TP * TP + i * TP + j];
  R[e] = s;
}

// Precision form: bfloat16 operands, float32 accumulation
// (v_mfma_f32_16x16x32_bf16: lane l supplies A[l%16][8(l/16) .. 8(l/16)+7] and
// B[8(l/16) .. +7][l%16]; component r of lane l is D[4(l/16) + r][l%16]).  The
// staged tile is [c][t][v] in bfloat16 (vertices contiguous), so both operands
// are one 16-byte LDS read per lane.  64 vertices per tile (two MFMA K steps).
constexpr int BF_VT = 64;
constexpr int BF_LD = BF_VT + 8;  // 16-byte aligned rows

typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef float f4v __attribute__((ext_vector_type(4)));

template <int TP>
__global__ void __launch_bounds__(AC_WAVES * 64)
k_autocorr_bf16(const float* __restrict__ frames, int n, int T, int nw, int P,
                float* __restrict__ part) {
  constexpr int NT = TP / 16;
  constexpr int JOBS = 3 * NT * (NT + 1) / 2;
  constexpr int JPW = (JOBS + AC_WAVES - 1) / AC_WAVES;
  __shared__ __attribute__((aligned(16))) __bf16 tile[3 * TP * BF_LD];
  const int p = blockIdx.x, w = blockIdx.y;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int per = (n + P - 1) / P;
  const int v_begin = p * per, v_end = min(n, v_begin + per);
  const float* base = frames + (size_t)w * T * 3 * n;
  f4v acc[JPW];
  int jc[JPW], ji[JPW], jj[JPW];
  for (int q = 0; q < JPW; ++q) {
    acc[q] = f4v{0.f, 0.f, 0.f, 0.f};
    const int job = wave + q * AC_WAVES;
    jc[q] = -1;
    if (job < JOBS) {
      const int per_c = NT * (NT + 1) / 2;
      jc[q] = job / per_c;
      int rem = job % per_c, bi = 0;
      while (rem >= NT - bi) {
        rem -= NT - bi;
        ++bi;
      }
      ji[q] = bi;
      jj[q] = bi + rem;
    }
  }
  for (int v0 = v_begin; v0 < v_end; v0 += BF_VT) {
    const int nv = min(BF_VT, v_end - v0);
    __syncthreads();
    for (int e = threadIdx.x; e < TP * 3 * BF_VT; e += AC_WAVES * 64) {
      const int t = e / (3 * BF_VT), rem = e % (3 * BF_VT);
      const int v = rem / 3, c = rem % 3;
      float val = 0.f;
      if (t < T && v < nv) val = base[(size_t)t * 3 * n + (size_t)(v0 + v) * 3 + c];
      tile[(c * TP + t) * BF_LD + v] = (__bf16)val;
    }
    __syncthreads();
    for (int q = 0; q < JPW; ++q) {
      if (jc[q] < 0) continue;
      const __bf16* tc = tile + jc[q] * TP * BF_LD;
      const int ra = ji[q] * 16 + lane % 16, rb = jj[q] * 16 + lane % 16;
#pragma unroll
      for (int kk = 0; kk < BF_VT; kk += 32) {
        const bf8v a = *(const bf8v*)&tc[ra * BF_LD + kk + 8 * (lane / 16)];
        const bf8v b = *(const bf8v*)&tc[rb * BF_LD + kk + 8 * (lane / 16)];
        acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[q], 0, 0, 0);
      }
    }
  }
  float* out = part + ((size_t)w * P + p) * 3 * TP * TP;
  for (int q = 0; q < JPW; ++q) {
    if (jc[q] < 0) continue;
    float* oc = out + (size_t)jc[q] * TP * TP;
    for (int r = 0; r < 4; ++r) {
      const int gi = ji[q] * 16 + 4 * (lane / 16) + r, gj = jj[q] * 16 + lane % 16;
      oc[gi * TP + gj] = acc[q][r];
      oc[gj * TP + gi] = acc[q][r];
    }
  }
}

int pad_T(int T) { return T <= 32 ? 32 : 64; }


constexpr int PJ_V = 64;  // vertices per projection block

// ---------------------------------------------------------------------------
// Fused encode: the projection of Eq. (9) computed straight from the frames,
// with the delta coordinates of Eq. (3-4) formed on the fly in LDS and never
// written to memory (the products are linear, so U~^T (L A^T)^T is the same
// operation; each delta is still formed by its ring sum first).  Block = 64
// vertices of one window; the window's frames go by tiles of PF_TT.  All
// four waves form a tile's delta coordinates (lane = vertex, one 12- or
// 24-byte xyz gather per ring member and frame, as k_delta), then waves 0-2
// project it (wave c = coordinate c, as k_project) while the next tile is
// being formed into the other LDS buffer.  Every delta is evaluated exactly
// as k_delta does and rounded to the frames' type, and the sums run over the
// frames in order as in k_project, so the coefficients are bit for bit those
// of the two-kernel path.
// ---------------------------------------------------------------------------
constexpr int PF_TT = 8;  // frames per delta tile

template <typename Real, int KMAX>
__global__ void __launch_bounds__(kBlock)
k_project_frames(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                 const double* __restrict__ wdeg, int uniform, int n, int T, int k,
                 const Real* __restrict__ frames, const double* __restrict__ u_tilde,
                 Real* __restrict__ Y, double* __restrict__ mm) {
  __shared__ Real Ut[3 * 64 * KMAX];
  __shared__ Real D[2][PF_TT][3][PJ_V];
  const int w = blockIdx.y, blk = blockIdx.x;
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  const double* ug = u_tilde + (size_t)w * 3 * T * k;
  for (int e = tid; e < 3 * T * k; e += kBlock) Ut[e] = (Real)ug[e];
  const int i = blk * PJ_V + lane;
  const bool valid = i < n;
  int e0 = 0, e1 = 0;
  double wi = 0.0;
  if (valid) {
    e0 = rowptr[i];
    e1 = rowptr[i + 1];
    wi = wdeg[i];
  }
  const int deg = e1 - e0;
  int nb[DMAX];
#pragma unroll
  for (int d = 0; d < DMAX; ++d) nb[d] = d < deg ? col[e0 + d] : (valid ? i : 0);
  const Real* fw = frames + (size_t)w * T * 3 * n;
  const size_t fs = (size_t)3 * n;
  // delta coordinates of tile `tile` into buffer `buf` (frames wave, wave + 4)
  auto delta_tile = [&](int tile, int buf) {
#pragma unroll
    for (int q = 0; q < PF_TT / 4; ++q) {
      const int tt = wave + 4 * q, t = tile * PF_TT + tt;
      Xyz<Real> o{(Real)0, (Real)0, (Real)0};
      if (valid && t < T) {
        const Xyz<Real>* fr = (const Xyz<Real>*)(fw + (size_t)t * fs);
        Xyz<Real> v[DMAX];
#pragma unroll
        for (int d = 0; d < DMAX; ++d) v[d] = fr[nb[d]];
        double sx = 0.0, sy = 0.0, sz = 0.0;
#pragma unroll
        for (int d = 0; d < DMAX; ++d)
          if (d < deg) {
            sx += (double)v[d].x;
            sy += (double)v[d].y;
            sz += (double)v[d].z;
          }
        for (int e = e0 + DMAX; e < e1; ++e) {
          const Xyz<Real> u = fr[col[e]];
          sx += (double)u.x;
          sy += (double)u.y;
          sz += (double)u.z;
        }
        const Xyz<Real> own = fr[i];
        o.x = (Real)(uniform ? (double)own.x - wi * sx : wi * (double)own.x - sx);
        o.y = (Real)(uniform ? (double)own.y - wi * sy : wi * (double)own.y - sy);
        o.z = (Real)(uniform ? (double)own.z - wi * sz : wi * (double)own.z - sz);
      }
      D[buf][tt][0][lane] = o.x;
      D[buf][tt][1][lane] = o.y;
      D[buf][tt][2][lane] = o.z;
    }
  };
  Real acc[KMAX];
#pragma unroll
  for (int r = 0; r < KMAX; ++r) acc[r] = 0;
  const int ntile = (T + PF_TT - 1) / PF_TT;
  delta_tile(0, 0);
  __syncthreads();
  const int c = wave;  // coordinate of waves 0-2 in the projection
  for (int tile = 0; tile < ntile; ++tile) {
    const int buf = tile & 1;
    if (tile + 1 < ntile) delta_tile(tile + 1, buf ^ 1);
    if (c < 3) {
      const Real* uc = Ut + c * T * k;
      for (int tt = 0; tt < PF_TT; ++tt) {
        const int t = tile * PF_TT + tt;
        if (t >= T) break;
        const Real d = D[buf][tt][c][lane];
#pragma unroll
        for (int r = 0; r < KMAX; ++r)
          if (r < k) acc[r] += uc[t * k + r] * d;
      }
    }
    __syncthreads();
  }
  if (c >= 3) return;
  Real* yw = Y + ((size_t)w * 3 + c) * k * n;
  const int nblk = gridDim.x;
  for (int r = 0; r < k; ++r) {
    if (valid) yw[(size_t)r * n + i] = acc[r];
    const double lo = wave_min(valid ? (double)acc[r] : 1e300);
    const double hi = wave_max(valid ? (double)acc[r] : -1e300);
    if (lane == 0) {
      double* o = mm + ((((size_t)w * 3 + c) * k + r) * nblk + blk) * 2;
      o[0] = lo;
      o[1] = hi;
    }
  }
}

__device__ inline uint16_t quant_code(double y, double lo, double hi, int bits) {
#pragma clang fp contract(off)
  const double levels = (double)((1 << bits) - 1);
  if (hi == lo) return 0;
  const double sc = levels / (hi - lo);
  const double t = (y - lo) * sc;
  double q = floor(t + 0.5);
  q = fmin(levels, fmax(0.0, q));
  return (uint16_t)q;
}

// Range of one row from the per-block partials, stored as float32 (rounded
// outwards for float64 data), then the row's codes (or raw values).
template <typename Real>
__global__ void __launch_bounds__(kBlock)
k_quantise_rows(const Real* __restrict__ Y, int n, int k, int nblk, const double* __restrict__ mm,
                int bits, uint8_t* records, size_t rec_bytes, size_t off_ranges, size_t off_codes) {
  __shared__ double slo[kBlock], shi[kBlock];
  const int row = blockIdx.y;  // (c, r) within the window
  const int w = blockIdx.z;
  const int c = row / k, r = row % k;
  uint8_t* rec = records + (size_t)w * rec_bytes;
  const Real* y = Y + (((size_t)w * 3 + c) * k + r) * n;
  const size_t code_base = ((size_t)c * k + r) * n;
  if (bits == 0) {
    Real* raw = (Real*)(rec + off_codes) + code_base;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) raw[i] = y[i];
    return;
  }
  const double* m = mm + ((((size_t)w * 3 + c) * k + r) * nblk) * 2;
  double lo = 1e300, hi = -1e300;
  for (int b = threadIdx.x; b < nblk; b += kBlock) {
    lo = fmin(lo, m[2 * b]);
    hi = fmax(hi, m[2 * b + 1]);
  }
  slo[threadIdx.x] = lo;
  shi[threadIdx.x] = hi;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      slo[threadIdx.x] = fmin(slo[threadIdx.x], slo[threadIdx.x + s]);
      shi[threadIdx.x] = fmax(shi[threadIdx.x], shi[threadIdx.x + s]);
    }
    __syncthreads();
  }
  const float flo = __double2float_rd(slo[0]);
  const float fhi = __double2float_ru(shi[0]);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    float* rg = (float*)(rec + off_ranges) + ((size_t)c * k + r) * 2;
    rg[0] = flo;
    rg[1] = fhi;
  }
  uint16_t* codes = (uint16_t*)(rec + off_codes) + code_base;
  const double dlo = (double)flo, dhi = (double)fhi;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock)
    codes[i] = quant_code((double)y[i], dlo, dhi, bits);
}

// ---------------------------------------------------------------------------
// Anchors (Eq. 12): values A_c[t][N_j] of one window and coordinate, range
// over all of them (float32, outward for float64 data), 16-bit (or `bits`)
// codes [c][t][j].
// ---------------------------------------------------------------------------
template <typename Real>
__global__ void __launch_bounds__(kBlock)
k_anchors(const Real* __restrict__ frames, int n, int T, const int32_t* __restrict__ anchors,
          int nc, int bits, uint8_t* records, size_t rec_bytes, size_t off_arange,
          size_t off_anchors) {
  __shared__ double slo[kBlock], shi[kBlock];
  const int w = blockIdx.x, c = blockIdx.y;
  const Real* fw = frames + (size_t)w * T * 3 * n;
  uint8_t* rec = records + (size_t)w * rec_bytes;
  const int m = T * nc;
  if (bits == 0) {
    Real* raw = (Real*)(rec + off_anchors) + (size_t)c * m;
    for (int e = threadIdx.x; e < m; e += kBlock) {
      const int t = e / nc, j = e % nc;
      raw[e] = fw[(size_t)t * 3 * n + 3 * (size_t)anchors[j] + c];
    }
    return;
  }
  double lo = 1e300, hi = -1e300;
  for (int e = threadIdx.x; e < m; e += kBlock) {
    const int t = e / nc, j = e % nc;
    const double v = (double)fw[(size_t)t * 3 * n + 3 * (size_t)anchors[j] + c];
    lo = fmin(lo, v);
    hi = fmax(hi, v);
  }
  slo[threadIdx.x] = lo;
  shi[threadIdx.x] = hi;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      slo[threadIdx.x] = fmin(slo[threadIdx.x], slo[threadIdx.x + s]);
      shi[threadIdx.x] = fmax(shi[threadIdx.x], shi[threadIdx.x + s]);
    }
    __syncthreads();
  }
  const float flo = __double2float_rd(slo[0]);
  const float fhi = __double2float_ru(shi[0]);
  if (threadIdx.x == 0) {
    float* rg = (float*)(rec + off_arange) + 2 * c;
    rg[0] = flo;
    rg[1] = fhi;
  }
  uint16_t* codes = (uint16_t*)(rec + off_anchors) + (size_t)c * m;
  for (int e = threadIdx.x; e < m; e += kBlock) {
    const int t = e / nc, j = e % nc;
    const double v = (double)fw[(size_t)t * 3 * n + 3 * (size_t)anchors[j] + c];
    codes[e] = quant_code(v, (double)flo, (double)fhi, bits);
  }
}

// The record header (the problem sizes and formats), and zeros in the
// alignment gaps after the header and after each section, so that every byte
// of a record is defined.
__global__ void k_header(uint8_t* rec, RecordLayout l) {
  int32_t* h = (int32_t*)rec;
  if (threadIdx.x == 0) {
    h[0] = kRecordMagic;
    h[1] = l.T;
    h[2] = l.k;
    h[3] = l.n;
    h[4] = l.nc;
    h[5] = l.coef_bits;
    h[6] = l.anchor_bits;
    h[7] = l.dict_bits;
    h[8] = l.precision;
    for (int i = 9; i < 16; ++i) h[i] = 0;
  }
  const size_t dict = (size_t)3 * l.T * l.k * (l.dict_bits > 0 ? 2 : l.real);
  const size_t codes = (size_t)3 * l.k * l.n * (l.coef_bits > 0 ? 2 : l.real);
  const size_t anchors = (size_t)3 * l.T * l.nc * (l.anchor_bits > 0 ? 2 : l.real);
  // (end of a section's data, start of the next section)
  const size_t gap[6][2] = {{64, l.off_dict},
                            {l.off_dict + dict, l.off_ranges},
                            {l.off_ranges + (size_t)3 * l.k * 2 * 4, l.off_codes},
                            {l.off_codes + codes, l.off_arange},
                            {l.off_arange + (size_t)3 * 2 * 4, l.off_anchors},
                            {l.off_anchors + anchors, l.bytes}};
  for (int g = 0; g < 6; ++g)
    for (size_t b = gap[g][0] + threadIdx.x; b < gap[g][1]; b += blockDim.x) rec[b] = 0;
}

}  // namespace

int autocorr_blocks(int n, int nw) {
  int P = (1024 + nw - 1) / nw;
  P = std::max(1, std::min(P, (n + AC_VT - 1) / AC_VT));
  return P;
}

void launch_delta(hipStream_t s, const MeshDev& m, const void* in, void* out, int32_t F,
                  int32_t precision, int fpb) {
  if (fpb < 1) fpb = 8;
  dim3 grid((m.n + kBlock - 1) / kBlock, (F + fpb - 1) / fpb);
  const int uni = m.laplacian == DMC_LAP_UNIFORM;
  prof::begin(s, DMC_KERNEL_DELTA);
  if (precision == DMC_FP64)
    hipLaunchKernelGGL(k_delta<double>, grid, dim3(kBlock), 0, s, m.rowptr, m.col, m.w64, uni,
                       m.n, F, fpb, (const double*)in, (double*)out);
  else
    hipLaunchKernelGGL(k_delta<float>, grid, dim3(kBlock), 0, s, m.rowptr, m.col, m.w64, uni,
                       m.n, F, fpb, (const float*)in, (float*)out);
  prof::end(s, DMC_KERNEL_DELTA);
}

// The autocorrelation is accumulated on the FP64 matrix cores for float32 and
// float64 frames alike: the eigenvalues of the uncentred R span many orders of
// magnitude (the mean shape dominates), and eigen-trajectories far below the
// largest one still carry delta-coordinate energy, so float32 accumulation would
// change the reconstruction measurably.
size_t autocorr_scratch_bytes(int32_t n, int32_t T, int32_t nw, int32_t precision, int P) {
  if (P < 1) P = autocorr_blocks(n, nw);
  const int TP = pad_T(T);
  return (size_t)nw * P * 3 * TP * TP * (precision == DMC_BF16 ? 4 : 8);
}

// precision form: bfloat16 products accumulated in float32, partials added in
// float64 in a fixed order
static void autocorr_bf16(hipStream_t s, const float* frames, int32_t n, int32_t T, int32_t nw,
                          float* part, double* R, int P) {
  dim3 grid(P, nw);
  const int tot = nw * 3 * T * T;
  dim3 rgrid((tot + kBlock - 1) / kBlock);
  prof::begin(s, DMC_KERNEL_AUTOCORR);
  if (T <= 32)
    hipLaunchKernelGGL((k_autocorr_bf16<32>), grid, dim3(AC_WAVES * 64), 0, s, frames, n, T, nw, P,
                       part);
  else
    hipLaunchKernelGGL((k_autocorr_bf16<64>), grid, dim3(AC_WAVES * 64), 0, s, frames, n, T, nw, P,
                       part);
  prof::end(s, DMC_KERNEL_AUTOCORR);
  if (T <= 32)
    hipLaunchKernelGGL((k_autocorr_reduce<float, 32>), rgrid, dim3(kBlock), 0, s,
                       (const float*)part, T, nw, P, R);
  else
    hipLaunchKernelGGL((k_autocorr_reduce<float, 64>), rgrid, dim3(kBlock), 0, s,
                       (const float*)part, T, nw, P, R);
}

template <typename In>
static void autocorr_impl(hipStream_t s, const In* frames, int32_t n, int32_t T, int32_t nw,
                          double* part, double* R, int P) {
  dim3 grid(P, nw);
  const int tot = nw * 3 * T * T;
  dim3 rgrid((tot + kBlock - 1) / kBlock);
  prof::begin(s, DMC_KERNEL_AUTOCORR);
  if (T <= 32)
    hipLaunchKernelGGL((k_autocorr<In, double, 32>), grid, dim3(AC_WAVES * 64), 0, s, frames, n,
                       T, nw, P, part);
  else
    hipLaunchKernelGGL((k_autocorr<In, double, 64>), grid, dim3(AC_WAVES * 64), 0, s, frames, n,
                       T, nw, P, part);
  prof::end(s, DMC_KERNEL_AUTOCORR);
  if (T <= 32)
    hipLaunchKernelGGL((k_autocorr_reduce<double, 32>), rgrid, dim3(kBlock), 0, s,
                       (const double*)part, T, nw, P, R);
  else
    hipLaunchKernelGGL((k_autocorr_reduce<double, 64>), rgrid, dim3(kBlock), 0, s,
                       (const double*)part, T, nw, P, R);
}

void launch_autocorr(hipStream_t s, const void* frames, int32_t n, int32_t T, int32_t nw,
                     int32_t precision, void* part, double* R, int P) {
  if (P < 1) P = autocorr_blocks(n, nw);
  P = std::min(P, std::max(1, n));
  if (precision == DMC_FP64)
    autocorr_impl(s, (const double*)frames, n, T, nw, (double*)part, R, P);
  else if (precision == DMC_BF16)
    autocorr_bf16(s, (const float*)frames, n, T, nw, (float*)part, R, P);
  else
    autocorr_impl(s, (const float*)frames, n, T, nw, (double*)part, R, P);
}

size_t project_scratch_bytes(int32_t n, int32_t T, int32_t k, int32_t nw, int32_t precision) {
  (void)T;
  const size_t nblk = (n + PJ_V - 1) / PJ_V;
  const size_t y = align_up((size_t)nw * 3 * k * n * (precision == DMC_FP64 ? 8 : 4));
  const size_t mm = align_up((size_t)nw * 3 * k * nblk * 2 * 8);
  return y + mm;
}

template <typename Real>
static void project_impl(hipStream_t s, const MeshDev& m, const void* frames, int32_t T,
                         int32_t k, int32_t nw, int32_t coef_bits, const double* u_tilde,
                         uint8_t* records, size_t rec_bytes, const RecordLayout& lay,
                         void* scratch, void* coef_out) {
  const int n = m.n;
  const int nblk = (n + PJ_V - 1) / PJ_V;
  Real* Y = coef_out ? (Real*)coef_out : (Real*)scratch;
  double* mm = (double*)((uint8_t*)scratch +
                         align_up((size_t)nw * 3 * k * n * sizeof(Real)));
  dim3 grid(nblk, nw);
  const int uni = m.laplacian == DMC_LAP_UNIFORM;
  const Real* fr = (const Real*)frames;
  prof::begin(s, DMC_KERNEL_PROJECT);
  if (k <= 8)
    hipLaunchKernelGGL((k_project_frames<Real, 8>), grid, dim3(kBlock), 0, s, m.rowptr, m.col,
                       m.w64, uni, n, T, k, fr, u_tilde, Y, mm);
  else if (k <= 16)
    hipLaunchKernelGGL((k_project_frames<Real, 16>), grid, dim3(kBlock), 0, s, m.rowptr, m.col,
                       m.w64, uni, n, T, k, fr, u_tilde, Y, mm);
  else
    hipLaunchKernelGGL((k_project_frames<Real, 32>), grid, dim3(kBlock), 0, s, m.rowptr, m.col,
                       m.w64, uni, n, T, k, fr, u_tilde, Y, mm);
  prof::end(s, DMC_KERNEL_PROJECT);
  const int chunks = std::max(1, std::min(64, (n + 4 * kBlock - 1) / (4 * kBlock)));
  dim3 qgrid(chunks, 3 * k, nw);
  prof::begin(s, DMC_KERNEL_QUANTISE);
  hipLaunchKernelGGL(k_quantise_rows<Real>, qgrid, dim3(kBlock), 0, s, (const Real*)Y, n, k,
                     nblk, (const double*)mm, coef_bits, records, rec_bytes, lay.off_ranges,
                     lay.off_codes);
  prof::end(s, DMC_KERNEL_QUANTISE);
}

void launch_project_quantise(hipStream_t s, const MeshDev& m, const void* frames, int32_t T,
                             int32_t k, int32_t nw, int32_t precision, int32_t coef_bits,
                             const double* u_tilde, uint8_t* records, size_t rec_bytes,
                             const RecordLayout& lay, void* scratch, void* coef_out) {
  if (precision == DMC_FP64)
    project_impl<double>(s, m, frames, T, k, nw, coef_bits, u_tilde, records, rec_bytes, lay,
                         scratch, coef_out);
  else
    project_impl<float>(s, m, frames, T, k, nw, coef_bits, u_tilde, records, rec_bytes, lay,
                        scratch, coef_out);
}

void launch_anchors(hipStream_t s, const MeshDev& m, const void* frames, int32_t T, int32_t nw,
                    int32_t precision, int32_t anchor_bits, uint8_t* records, size_t rec_bytes,
                    const RecordLayout& lay) {
  dim3 grid(nw, 3);
  prof::begin(s, DMC_KERNEL_ANCHORS);
  if (precision == DMC_FP64)
    hipLaunchKernelGGL(k_anchors<double>, grid, dim3(kBlock), 0, s, (const double*)frames, m.n,
                       T, m.anchors, m.nc, anchor_bits, records, rec_bytes, lay.off_arange,
                       lay.off_anchors);
  else
    hipLaunchKernelGGL(k_anchors<float>, grid, dim3(kBlock), 0, s, (const float*)frames, m.n, T,
                       m.anchors, m.nc, anchor_bits, records, rec_bytes, lay.off_arange,
                       lay.off_anchors);
  prof::end(s, DMC_KERNEL_ANCHORS);
}

void launch_write_header(hipStream_t s, uint8_t* rec, const RecordLayout& l) {
  hipLaunchKernelGGL(k_header, dim3(1), dim3(64), 0, s, rec, l);
}

}  // namespace dmc
