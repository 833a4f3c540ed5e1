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
  // element (t, v, c) of a vertex tile -> tile[c][v][t] (zero padding); the
  // next tile's loads are in flight in registers while the current one is
  // multiplied
  constexpr int PER = TP * 3 * AC_VT / (AC_WAVES * 64);
  static_assert(TP * 3 * AC_VT % (AC_WAVES * 64) == 0, "whole elements per thread");
  In nxt[PER];
  auto load = [&](int v0) {
    const int nv = min(AC_VT, v_end - v0);
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = threadIdx.x + u * AC_WAVES * 64;
      const int t = e / (3 * AC_VT), rem = e % (3 * AC_VT);
      const int v = rem / 3, c = rem % 3;
      nxt[u] = (t < T && v < nv) ? base[(size_t)t * 3 * n + (size_t)(v0 + v) * 3 + c] : (In)0;
    }
  };
  if (v_begin < v_end) load(v_begin);
  for (int v0 = v_begin; v0 < v_end; v0 += AC_VT) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = threadIdx.x + u * AC_WAVES * 64;
      const int t = e / (3 * AC_VT), rem = e % (3 * AC_VT);
      const int v = rem / 3, c = rem % 3;
      tile[(c * AC_VT + v) * LD + t] = (Real)nxt[u];
    }
    __syncthreads();
    if (v0 + AC_VT < v_end) load(v0 + AC_VT);
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

// R entry e = sum over the P partials: block = 64 consecutive entries (lane
// = entry, so every load is coalesced), wave g adding the partials p = g,
// g + 4, ... in order, the four wave sums added as (s0 + s1) + (s2 + s3)
// (deterministic; four times the parallelism of one thread per entry).
template <typename Real, int TP>
__global__ void __launch_bounds__(kBlock)
k_autocorr_reduce(const Real* __restrict__ part, int T, int nw, int P, double* __restrict__ R) {
  constexpr int NW = kBlock / 64;
  __shared__ double sh[NW][64];
  const int lane = threadIdx.x % 64, g = threadIdx.x / 64;
  const int e = blockIdx.x * 64 + lane;
  const int per_w = 3 * T * T;
  double s = 0.0;
  if (e < nw * per_w) {
    const int w = e / per_w, rem = e % per_w;
    const int c = rem / (T * T), ij = rem % (T * T);
    const int i = ij / T, j = ij % T;
    const Real* pe = part + (((size_t)w * P) * 3 + c) * TP * TP + i * TP + j;
    const size_t stride = (size_t)3 * TP * TP;
    for (int p = g; p < P; p += NW) s += (double)pe[(size_t)p * stride];
  }
  sh[g][lane] = s;
  __syncthreads();
  if (g == 0 && e < nw * per_w) R[e] = (sh[0][lane] + sh[1][lane]) + (sh[2][lane] + sh[3][lane]);
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
  // the next tile's loads are in flight in registers while the current one
  // is multiplied
  constexpr int PER = TP * 3 * BF_VT / (AC_WAVES * 64);
  static_assert(TP * 3 * BF_VT % (AC_WAVES * 64) == 0, "whole elements per thread");
  float nxt[PER];
  auto load = [&](int v0) {
    const int nv = min(BF_VT, v_end - v0);
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = threadIdx.x + u * AC_WAVES * 64;
      const int t = e / (3 * BF_VT), rem = e % (3 * BF_VT);
      const int v = rem / 3, c = rem % 3;
      nxt[u] = (t < T && v < nv) ? base[(size_t)t * 3 * n + (size_t)(v0 + v) * 3 + c] : 0.f;
    }
  };
  if (v_begin < v_end) load(v_begin);
  for (int v0 = v_begin; v0 < v_end; v0 += BF_VT) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = threadIdx.x + u * AC_WAVES * 64;
      const int t = e / (3 * BF_VT), rem = e % (3 * BF_VT);
      const int v = rem / 3, c = rem % 3;
      tile[(c * TP + t) * BF_LD + v] = (__bf16)nxt[u];
    }
    __syncthreads();
    if (v0 + BF_VT < v_end) load(v0 + BF_VT);
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
// project it (wave c = coordinate c, as k_project).  The gathers of the next
// tile (every ring member and the vertex itself, both of a wave's frames)
// are issued together before the current tile is projected, so their
// latency hides behind the products instead of following one another.
// Every delta is evaluated exactly as k_delta does and rounded to the
// frames' type, and the sums run over the frames in order as in k_project,
// so the coefficients are bit for bit those of the two-kernel path.
// ---------------------------------------------------------------------------
constexpr int PF_TT = 8;  // frames per delta tile
constexpr int PF_FQ = PF_TT / (kBlock / 64);  // frames per wave and tile
// ring members held in registers (valence 6 is the rule on these meshes: a
// larger pad would add gathers of the vertex itself; longer rings finish
// from memory)
constexpr int PF_DMAX = 6;

template <typename Real, int KMAX>
__global__ void __launch_bounds__(kBlock)
k_project_frames(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                 const double* __restrict__ wdeg, int uniform, int n, int T, int k,
                 const Real* __restrict__ frames, const double* __restrict__ u_tilde,
                 Real* __restrict__ Y, double* __restrict__ mm) {
  // the dictionary with rows padded to KMAX by zeros: a frame's row is read
  // as whole 16-byte words
  __shared__ __align__(16) Real Ut[3 * 64 * KMAX];
  __shared__ Real D[2][PF_TT][3][PJ_V];
  const int w = blockIdx.y, blk = blockIdx.x;
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  const double* ug = u_tilde + (size_t)w * 3 * T * k;
  for (int e = tid; e < 3 * T * KMAX; e += kBlock) {
    const int r = e % KMAX, ct = e / KMAX;
    Ut[e] = r < k ? (Real)ug[(size_t)ct * k + r] : (Real)0;
  }
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
  const int iv = valid ? i : 0;
  int nb[PF_DMAX];
#pragma unroll
  for (int d = 0; d < PF_DMAX; ++d) nb[d] = d < deg ? col[e0 + d] : iv;
  const Real* fw = frames + (size_t)w * T * 3 * n;
  const size_t fs = (size_t)3 * n;
  // the wave's gathers of tile `tile`: ring members, then the vertex itself
  Xyz<Real> g[PF_FQ][PF_DMAX + 1];
  auto gather = [&](int tile) {
#pragma unroll
    for (int q = 0; q < PF_FQ; ++q) {
      const int t = min(tile * PF_TT + wave + 4 * q, T - 1);
      const Xyz<Real>* fr = (const Xyz<Real>*)(fw + (size_t)t * fs);
#pragma unroll
      for (int d = 0; d < PF_DMAX; ++d) g[q][d] = fr[nb[d]];
      g[q][PF_DMAX] = fr[iv];
    }
  };
  // delta coordinates of tile `tile` from the gathers into buffer `buf`
  // (pads beyond the ring add exact zeros: a sum that starts at +0 is never
  // -0, so the sums are those of the ring alone)
  auto delta_store = [&](int tile, int buf) {
#pragma unroll
    for (int q = 0; q < PF_FQ; ++q) {
      const int tt = wave + 4 * q, t = tile * PF_TT + tt;
      double sx = 0.0, sy = 0.0, sz = 0.0;
#pragma unroll
      for (int d = 0; d < PF_DMAX; ++d) {
        const bool in = d < deg;
        sx += in ? (double)g[q][d].x : 0.0;
        sy += in ? (double)g[q][d].y : 0.0;
        sz += in ? (double)g[q][d].z : 0.0;
      }
      if (deg > PF_DMAX) {
        const Xyz<Real>* fr = (const Xyz<Real>*)(fw + (size_t)min(t, T - 1) * fs);
        for (int e = e0 + PF_DMAX; e < e1; ++e) {
          const Xyz<Real> u = fr[col[e]];
          sx += (double)u.x;
          sy += (double)u.y;
          sz += (double)u.z;
        }
      }
      const Xyz<Real> own = g[q][PF_DMAX];
      Xyz<Real> o{(Real)0, (Real)0, (Real)0};
      if (valid && t < T) {
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
  gather(0);
  delta_store(0, 0);
  __syncthreads();
  const int c = wave;  // coordinate of waves 0-2 in the projection
  for (int tile = 0; tile < ntile; ++tile) {
    const int buf = tile & 1;
    const bool more = tile + 1 < ntile;
    if (more) gather(tile + 1);
    if (c < 3) {
      const Real* uc = Ut + c * T * KMAX;
#pragma unroll
      for (int tt = 0; tt < PF_TT; ++tt) {
        const int t = tile * PF_TT + tt;
        if (t >= T) break;
        const Real d = D[buf][tt][c][lane];
#pragma unroll
        for (int r = 0; r < KMAX; ++r) acc[r] += uc[t * KMAX + r] * d;
      }
    }
    if (more) delta_store(tile + 1, buf ^ 1);
    __syncthreads();
  }
  if (c >= 3) return;
  Real* yw = Y + ((size_t)w * 3 + c) * k * n;
  const int nblk = gridDim.x;
  // the coefficients pass through the dictionary's LDS (idle after the last
  // barrier), each lane reading back only its own: the loop over the k rows
  // then indexes LDS, and acc keeps static indices (a runtime index would
  // move it to scratch memory)
  static_assert(3 * KMAX * PJ_V <= 3 * 64 * KMAX, "coefficients fit the dictionary's LDS");
  Real* keep = Ut + (size_t)c * KMAX * PJ_V;
#pragma unroll
  for (int r = 0; r < KMAX; ++r) keep[r * PJ_V + lane] = acc[r];
  for (int r = 0; r < k; ++r) {
    const Real a = keep[r * PJ_V + lane];
    if (valid) yw[(size_t)r * n + i] = a;
    const double lo = wave_min(valid ? (double)a : 1e300);
    const double hi = wave_max(valid ? (double)a : -1e300);
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

// ---------------------------------------------------------------------------
// The record (layout in dmc.h): packed segments of codes, their tables, the
// header.  Codes are Eq. (10)'s, with per-segment bit widths: the dictionary
// at dict_bits over [-1, 1] (plain) or per column over its own range as
// values or as the difference from the previous window's column, whichever
// needs fewer bits at a step no coarser than the plain code's (Sec. IV,
// Fig. 6); the coefficient rows at coef_bits, or with the fewest bits that
// keep a caller-given step (Fig. 5); the anchors at anchor_bits.
// ---------------------------------------------------------------------------

// fewest bits b in 1..cap with (hi - lo) <= step (2^b - 1), cap if none; 0
// for an empty range
__device__ inline uint32_t bits_for_step(double lo, double hi, double step, uint32_t cap) {
#pragma clang fp contract(off)
  const double width = hi - lo;
  if (width == 0.0) return 0;
  const double ratio = width / step;
  for (uint32_t b = 1; b < cap; ++b)
    if ((double)((1u << b) - 1u) >= ratio) return b;
  return cap;
}

__device__ inline double dequant_code(uint32_t code, double lo, double hi, int bits) {
#pragma clang fp contract(off)
  const double levels = (double)((1u << bits) - 1u);
  const double step = (hi - lo) / levels;
  return lo + (double)code * step;
}

// OR of the codes of a packed segment that fall in its 32-bit word wi; code(j)
// gives code j (j < count)
template <typename CodeOf>
__device__ inline uint32_t pack_word(uint32_t wi, uint32_t count, uint32_t bits, CodeOf code) {
  const uint64_t b0 = (uint64_t)wi * 32;
  uint32_t j = (uint32_t)(b0 / bits);
  uint64_t word = 0;
  for (; j < count && (uint64_t)j * bits < b0 + 32; ++j) {
    const int64_t pos = (int64_t)j * bits - (int64_t)b0;
    const uint64_t c = code(j);
    word |= pos >= 0 ? c << pos : c >> (-pos);
  }
  return (uint32_t)word;
}

// Header words: sizes and formats; the words filled later (has_diff,
// used bytes, dictionary words) start at zero.  Zeros in the alignment
// gaps of the fixed part, so every byte of a record's stream is defined.
// block w: the header of record w (records rec_bytes apart) and its alignment gaps
__global__ void k_header(uint8_t* records, size_t rec_bytes, RecordLayout l) {
  uint8_t* rec = records + (size_t)blockIdx.x * rec_bytes;
  int32_t* h = (int32_t*)rec;
  if (threadIdx.x < kHeaderBytes / 4) {
    const int i = threadIdx.x;
    int32_t v = 0;
    switch (i) {
      case kHdrMagic: v = kRecordMagic; break;
      case kHdrT: v = l.T; break;
      case kHdrK: v = l.k; break;
      case kHdrN: v = l.n; break;
      case kHdrNc: v = l.nc; break;
      case kHdrCoefBits: v = l.coef_bits; break;
      case kHdrAnchorBits: v = l.anchor_bits; break;
      case kHdrDictBits: v = l.dict_bits; break;
      case kHdrPrecision: v = l.precision; break;
      case kHdrDictMode: v = l.dict_mode; break;
      case kHdrStepLo: v = (int32_t)(uint32_t)__double_as_longlong(l.coef_step); break;
      case kHdrStepHi: v = (int32_t)(uint32_t)((uint64_t)__double_as_longlong(l.coef_step) >> 32); break;
      default: v = 0;
    }
    h[i] = v;
  }
  const size_t gap[2][2] = {{l.off_arange + 3 * 8, l.off_anchors},
                            {l.off_anchors + 3 * l.anchor_seg, l.off_var}};
  for (int g = 0; g < 2; ++g)
    for (size_t b = gap[g][0] + threadIdx.x; b < gap[g][1]; b += blockDim.x) rec[b] = 0;
}

// Dictionary coder: one block (4 waves) per group of windows; wave v codes
// the columns q = v, v + 4, ... (q = c k + j) of each window, one lane per
// frame.  With differences allowed the windows run in order in one block
// (each column may refer to the previous window's dequantised column);
// otherwise every window has a block of its own.  Writes the dequantised
// dictionary u_tilde [nw][3][T][k], the column table and the packed
// segments (or raw values) of each record, and the header's dictionary words
// and difference flag.
constexpr int DC_COLS = 96;  // 3 k, k <= 32

template <typename Real>
__global__ void __launch_bounds__(kBlock)
k_dict_code(const double* __restrict__ u_canon, int nw, int per_block, RecordLayout l,
            uint8_t* records, size_t rec_bytes, double* __restrict__ u_tilde) {
  __shared__ uint16_t sc[DC_COLS][64];
  __shared__ uint32_t sbits[DC_COLS], smode[DC_COLS];
  const int T = l.T, k = l.k, nq = 3 * k;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int db = l.dict_bits;
  const double step = db > 0 ? 2.0 / (double)((1u << db) - 1u) : 0.0;
  const int w0 = blockIdx.x * per_block, w1 = min(nw, w0 + per_block);
  for (int w = w0; w < w1; ++w) {
    uint8_t* rec = records + (size_t)w * rec_bytes;
    SegEntry* tab = (SegEntry*)(rec + l.off_dtab);
    const double* U = u_canon + (size_t)w * 3 * T * k;
    double* Ut = u_tilde + (size_t)w * 3 * T * k;
    const double* Up = w > w0 ? u_tilde + (size_t)(w - 1) * 3 * T * k : nullptr;
    for (int q = wave; q < nq; q += kBlock / 64) {
      const int c = q / k, j = q % k, t = lane;
      const bool valid = t < T;
      const size_t at = ((size_t)c * T + t) * k + j;
      const double u = valid ? U[at] : 0.0;
      double lo = -1.0, hi = 1.0, ut = u;
      uint32_t bits = db, mode = 0, code = 0;
      if (db == 0) {
        ut = (double)(Real)u;  // raw values in the frames' type
        lo = hi = 0.0;
      } else if (l.dict_mode == 0) {
        code = quant_code(u, -1.0, 1.0, db);
        ut = dequant_code(code, -1.0, 1.0, db);
      } else {
        // values: their own range, the fewest bits at the plain code's step
        const double la = (double)__double2float_rd(wave_min(valid ? u : 1e300));
        const double ha = (double)__double2float_ru(wave_max(valid ? u : -1e300));
        const uint32_t ba = bits_for_step(la, ha, step, 16);
        lo = la;
        hi = ha;
        bits = ba;
        double val = u;
        if (Up) {
          const double pu = valid ? Up[at] : 0.0;
          const double d = u - pu;
          const double ld = (double)__double2float_rd(wave_min(valid ? d : 1e300));
          const double hd = (double)__double2float_ru(wave_max(valid ? d : -1e300));
          const uint32_t bd = bits_for_step(ld, hd, step, 16);
          if (bd < ba) {
            lo = ld;
            hi = hd;
            bits = bd;
            mode = 1;
            val = d;
          }
        }
        code = bits ? quant_code(val, lo, hi, bits) : 0u;
        const double deq = bits ? dequant_code(code, lo, hi, bits) : lo;
        ut = mode ? Up[at] + deq : deq;
      }
      if (valid) {
        Ut[at] = ut;
        sc[q][t] = (uint16_t)code;
      }
      if (lane == 0) {
        tab[q].lo = (float)lo;
        tab[q].hi = (float)hi;
        tab[q].bits_mode = bits | (mode << 8);
        sbits[q] = bits;
        smode[q] = mode;
      }
      // raw values go straight into the segment below, once offsets are known
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t off = 0, diff = 0;
      for (int q = 0; q < nq; ++q) {
        tab[q].word_off = off;
        off += seg_words(T, sbits[q], (uint32_t)l.real);
        diff |= smode[q];
      }
      int32_t* h = (int32_t*)rec;
      h[kHdrDictWords] = (int32_t)off;
      h[kHdrHasDiff] = (int32_t)diff;
    }
    __syncthreads();
    uint32_t* var = (uint32_t*)(rec + l.off_var);
    for (int q = wave; q < nq; q += kBlock / 64) {
      const uint32_t bits = sbits[q];
      uint32_t* seg = var + tab[q].word_off;
      const uint32_t nwd = seg_words(T, bits, (uint32_t)l.real);
      if (db == 0) {
        const int c = q / k, j = q % k;
        Real* raw = (Real*)seg;
        if (lane < T) raw[lane] = (Real)U[((size_t)c * T + lane) * k + j];
        // the padding of the segment: bytes after T raw values up to nwd words
        for (uint32_t b = (uint32_t)(T * sizeof(Real)) + lane; b < 4 * nwd; b += 64)
          ((uint8_t*)seg)[b] = 0;
      } else {
        for (uint32_t wi = lane; wi < nwd; wi += 64)
          seg[wi] = pack_word(wi, (uint32_t)T, bits, [&](uint32_t j) { return (uint32_t)sc[q][j]; });
      }
    }
    __syncthreads();
  }
}

// Coefficient-row ranges (block = one row q of one window w): the row's
// per-block partials from the projection reduced, rounded outwards to
// float32, and the row's bits (coef_bits, or the fewest for coef_step).
__global__ void __launch_bounds__(64)
k_row_range(int nblk, const double* __restrict__ mm, RecordLayout l, uint8_t* records,
            size_t rec_bytes) {
  const int q = blockIdx.x, w = blockIdx.y, nq = 3 * l.k, lane = threadIdx.x;
  SegEntry* tab = (SegEntry*)(records + (size_t)w * rec_bytes + l.off_rtab);
  const double* m = mm + ((size_t)w * nq + q) * nblk * 2;
  double lo = 1e300, hi = -1e300;
  for (int b = lane; b < nblk; b += 64) {
    lo = fmin(lo, m[2 * b]);
    hi = fmax(hi, m[2 * b + 1]);
  }
  lo = wave_min(lo);
  hi = wave_max(hi);
  const float flo = __double2float_rd(lo), fhi = __double2float_ru(hi);
  uint32_t bits = (uint32_t)l.coef_bits;
  if (l.coef_bits > 0 && l.coef_step > 0.0)
    bits = bits_for_step((double)flo, (double)fhi, l.coef_step, (uint32_t)l.coef_bits);
  if (lane == 0) {
    tab[q].lo = l.coef_bits > 0 ? flo : 0.f;
    tab[q].hi = l.coef_bits > 0 ? fhi : 0.f;
    tab[q].bits_mode = bits;
  }
}

// Codes of the coefficient rows (Eq. 10) packed into their segments: block
// (x, q, w) packs a contiguous share of the words of row q of window w in
// rounds of kBlock words.  A round's codes are formed once each into LDS
// from coalesced loads (QP_U per thread, none behind a branch, so all are
// in flight at once), then thread t assembles word t of the round from the
// codes that fall in it.  A single-valued row (0 bits) keeps its raw-sized
// segment of zeros; raw rows are copied.  Each wave finds the row's word
// offset (after the dictionary segments) from the bits of the rows before
// it, lane r taking rows r and r + 64; block (0, q, w) stores it in the
// table and block (0, last row, w) the record's used bytes in the header.
constexpr int QP_U = 4;  // code loads per thread and pass of a round
template <typename Real>
__global__ void __launch_bounds__(kBlock)
k_quantise_pack(const Real* __restrict__ Y, int n, int k, RecordLayout l, uint8_t* records,
                size_t rec_bytes) {
  const int q = blockIdx.y, w = blockIdx.z, nq = 3 * k, lane = threadIdx.x % 64;
  uint8_t* rec = records + (size_t)w * rec_bytes;
  SegEntry* tab = (SegEntry*)(rec + l.off_rtab);
  uint32_t part = 0;
  for (int r = lane; r < q; r += 64)
    part += seg_words((uint32_t)n, tab[r].bits_mode & 0xff, (uint32_t)l.real);
  // (a sum of word counts, exact in float64)
  const uint32_t off = (uint32_t)((const int32_t*)rec)[kHdrDictWords] + (uint32_t)wave_sum((double)part);
  const SegEntry e = tab[q];
  const uint32_t bits = e.bits_mode & 0xff;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    tab[q].word_off = off;
    if (q == nq - 1) {
      const uint64_t used = l.off_var + 4ull * (off + seg_words((uint32_t)n, bits, (uint32_t)l.real));
      int32_t* hw = (int32_t*)rec;
      hw[kHdrUsedLo] = (int32_t)(uint32_t)used;
      hw[kHdrUsedHi] = (int32_t)(uint32_t)(used >> 32);
    }
  }
  const Real* y = Y + ((size_t)w * 3 * k + q) * n;
  uint32_t* seg = (uint32_t*)(rec + l.off_var) + off;
  const uint32_t stride = gridDim.x * kBlock;
  if (l.coef_bits == 0) {
    Real* raw = (Real*)seg;
    for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < (uint32_t)n; i += stride) raw[i] = y[i];
    const uint32_t nwd = seg_words((uint32_t)n, 0, sizeof(Real));
    for (uint32_t b = (uint32_t)n * sizeof(Real) + blockIdx.x * kBlock + threadIdx.x; b < 4 * nwd;
         b += stride)
      ((uint8_t*)seg)[b] = 0;
    return;
  }
  const uint32_t nwd = seg_words((uint32_t)n, bits, 4);
  if (bits == 0) {
    for (uint32_t wi = blockIdx.x * kBlock + threadIdx.x; wi < nwd; wi += stride) seg[wi] = 0u;
    return;
  }
  // a round holds at most 32 kBlock / bits + 1 codes; the passes store whole
  // QP_U kBlock slices (the entries beyond the round's codes are never read)
  __shared__ uint16_t cs[32 * kBlock + QP_U * kBlock];
  const double lo = (double)e.lo, hi = (double)e.hi;
  const uint32_t per = (nwd + gridDim.x - 1) / gridDim.x;
  const uint32_t wb = blockIdx.x * per, we = min(nwd, wb + per);
  for (uint32_t r0 = wb; r0 < we; r0 += kBlock) {
    const uint32_t rw = min((uint32_t)kBlock, we - r0);
    const uint32_t jlo = (uint32_t)((32ull * r0) / bits);
    const uint64_t jend = (32ull * (r0 + rw) + bits - 1) / bits;  // codes starting in the round
    const uint32_t jhi = (uint32_t)min((uint64_t)n, jend);
    const uint32_t nc = jhi > jlo ? jhi - jlo : 0u;
    for (uint32_t b = threadIdx.x; b < nc; b += QP_U * kBlock) {
      Real v[QP_U];
#pragma unroll
      for (int u = 0; u < QP_U; ++u) v[u] = y[min(jlo + b + u * kBlock, jhi - 1)];
#pragma unroll
      for (int u = 0; u < QP_U; ++u)
        cs[b + u * kBlock] = (uint16_t)quant_code((double)v[u], lo, hi, (int)bits);
    }
    __syncthreads();
    if (threadIdx.x < rw)
      seg[r0 + threadIdx.x] = pack_word(r0 + threadIdx.x, (uint32_t)n, bits,
                                        [&](uint32_t j) { return (uint32_t)cs[j - jlo]; });
    __syncthreads();
  }
}

// zeros from the record's used bytes to its capacity (a record's stream is
// its first used bytes; the rest of its slot is defined too)
__global__ void __launch_bounds__(kBlock)
k_zero_tail(uint8_t* records, size_t rec_bytes) {
  uint8_t* rec = records + (size_t)blockIdx.y * rec_bytes;
  const int32_t* h = (const int32_t*)rec;
  const uint64_t used = (uint64_t)(uint32_t)h[kHdrUsedLo] | ((uint64_t)(uint32_t)h[kHdrUsedHi] << 32);
  uint2* p = (uint2*)(rec + used);
  const size_t count = (rec_bytes - used) / 8;
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < count; i += (size_t)gridDim.x * kBlock)
    p[i] = make_uint2(0u, 0u);
}

// ---------------------------------------------------------------------------
// Anchors (Eq. 12): values A_c[t][N_a] of one window and coordinate, range
// over all of them (float32, rounded outwards), codes of anchor_bits packed
// in order j = t n_c + a (or raw values).  Two launches: partial extrema per
// chunk of values, then every block takes the range from the partials (the
// same bits in all of them) and packs its share of the segment's words.
// ---------------------------------------------------------------------------
constexpr int AN_CHUNKS = 32;

template <typename Real>
__device__ inline Real anchor_value(const Real* __restrict__ fw, int n, int nc,
                                    const int32_t* __restrict__ anchors, int c, int e) {
  const int t = e / nc, j = e % nc;
  return fw[(size_t)t * 3 * n + 3 * (size_t)anchors[j] + c];
}

template <typename Real>
__global__ void __launch_bounds__(kBlock)
k_anchor_minmax(const Real* __restrict__ frames, int n, int T, const int32_t* __restrict__ anchors,
                int nc, double* __restrict__ part) {
  __shared__ double slo[kBlock], shi[kBlock];
  const int ch = blockIdx.x, c = blockIdx.y, w = blockIdx.z;
  const Real* fw = frames + (size_t)w * T * 3 * n;
  const int m = T * nc, per = (m + AN_CHUNKS - 1) / AN_CHUNKS;
  const int e0 = ch * per, e1 = min(m, e0 + per);
  double lo = 1e300, hi = -1e300;
  for (int e = e0 + threadIdx.x; e < e1; e += kBlock) {
    const double v = (double)anchor_value(fw, n, nc, anchors, c, e);
    lo = fmin(lo, v);
    hi = fmax(hi, v);
  }
  slo[threadIdx.x] = lo;
  shi[threadIdx.x] = hi;
  __syncthreads();
  for (int st = kBlock / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) {
      slo[threadIdx.x] = fmin(slo[threadIdx.x], slo[threadIdx.x + st]);
      shi[threadIdx.x] = fmax(shi[threadIdx.x], shi[threadIdx.x + st]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double* o = part + (((size_t)w * 3 + c) * AN_CHUNKS + ch) * 2;
    o[0] = slo[0];
    o[1] = shi[0];
  }
}

template <typename Real>
__global__ void __launch_bounds__(kBlock)
k_anchor_pack(const Real* __restrict__ frames, int n, int T, const int32_t* __restrict__ anchors,
              int nc, int bits, const double* __restrict__ part, uint8_t* records,
              size_t rec_bytes, RecordLayout l) {
  const int c = blockIdx.y, w = blockIdx.z;
  const Real* fw = frames + (size_t)w * T * 3 * n;
  uint8_t* rec = records + (size_t)w * rec_bytes;
  const int m = T * nc;
  uint32_t* seg = (uint32_t*)(rec + l.off_anchors + (size_t)c * l.anchor_seg);
  float* rg = (float*)(rec + l.off_arange) + 2 * c;
  const uint32_t stride = gridDim.x * kBlock, first = blockIdx.x * kBlock + threadIdx.x;
  if (bits == 0) {
    Real* raw = (Real*)seg;
    for (uint32_t e = first; e < (uint32_t)m; e += stride)
      raw[e] = anchor_value(fw, n, nc, anchors, c, (int)e);
    for (size_t b = (size_t)m * sizeof(Real) + first; b < l.anchor_seg; b += stride)
      ((uint8_t*)seg)[b] = 0;
    if (first == 0) rg[0] = rg[1] = 0.f;
    return;
  }
  // the range: every lane adds the partials in the same order
  const double* pp = part + ((size_t)w * 3 + c) * AN_CHUNKS * 2;
  double lo = 1e300, hi = -1e300;
  for (int q = 0; q < AN_CHUNKS; ++q) {
    lo = fmin(lo, pp[2 * q]);
    hi = fmax(hi, pp[2 * q + 1]);
  }
  const float flo = __double2float_rd(lo), fhi = __double2float_ru(hi);
  if (first == 0) {
    rg[0] = flo;
    rg[1] = fhi;
  }
  const uint32_t nwd = (uint32_t)(l.anchor_seg / 4);
  for (uint32_t wi = first; wi < nwd; wi += stride)
    seg[wi] = pack_word(wi, (uint32_t)m, (uint32_t)bits, [&](uint32_t j) {
      return (uint32_t)quant_code((double)anchor_value(fw, n, nc, anchors, c, (int)j), (double)flo,
                                  (double)fhi, bits);
    });
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
  dim3 rgrid((tot + 63) / 64);
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
  dim3 rgrid((tot + 63) / 64);
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


template <typename Real>
static void project_impl(hipStream_t s, const MeshDev& m, const void* frames, int32_t T,
                         int32_t k, int32_t nw, const double* u_tilde, uint8_t* records,
                         size_t rec_bytes, const RecordLayout& lay, void* scratch,
                         void* coef_out) {
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
  prof::begin(s, DMC_KERNEL_QUANTISE);
  hipLaunchKernelGGL(k_row_range, dim3(3 * k, nw), dim3(64), 0, s, nblk, (const double*)mm, lay,
                     records, rec_bytes);
  // words of a row at its widest, spread so that a block writes a few per thread
  const uint32_t wmax = seg_words((uint32_t)n, lay.coef_bits > 0 ? lay.coef_bits : 0,
                                  (uint32_t)sizeof(Real));
  const int chunks = std::max(1, std::min(64, (int)((wmax + 16 * kBlock - 1) / (16 * kBlock))));
  hipLaunchKernelGGL(k_quantise_pack<Real>, dim3(chunks, 3 * k, nw), dim3(kBlock), 0, s,
                     (const Real*)Y, n, k, lay, records, rec_bytes);
  prof::end(s, DMC_KERNEL_QUANTISE);
}

size_t project_scratch_bytes(int32_t n, int32_t T, int32_t k, int32_t nw, int32_t precision) {
  (void)T;
  const size_t nblk = (n + PJ_V - 1) / PJ_V;
  const size_t y = align_up((size_t)nw * 3 * k * n * (precision == DMC_FP64 ? 8 : 4));
  const size_t mm = align_up((size_t)nw * 3 * k * nblk * 2 * 8);
  return y + mm;
}

void launch_project_quantise(hipStream_t s, const MeshDev& m, const void* frames, int32_t T,
                             int32_t k, int32_t nw, int32_t precision, const double* u_tilde,
                             uint8_t* records, size_t rec_bytes, const RecordLayout& lay,
                             void* scratch, void* coef_out) {
  if (precision == DMC_FP64)
    project_impl<double>(s, m, frames, T, k, nw, u_tilde, records, rec_bytes, lay, scratch,
                         coef_out);
  else
    project_impl<float>(s, m, frames, T, k, nw, u_tilde, records, rec_bytes, lay, scratch,
                        coef_out);
}

size_t anchors_scratch_bytes(int32_t nw) { return align_up((size_t)nw * 3 * AN_CHUNKS * 2 * 8); }

void launch_anchors(hipStream_t s, const MeshDev& m, const void* frames, int32_t T, int32_t nw,
                    int32_t precision, uint8_t* records, size_t rec_bytes, const RecordLayout& lay,
                    double* part) {
  const int mvals = T * m.nc;
  const uint32_t nwd = (uint32_t)(lay.anchor_seg / 4);
  const int pk = std::max(1, std::min(64, (int)((std::max<uint32_t>(nwd, mvals) + 4 * kBlock - 1) /
                                                (4 * kBlock))));
  prof::begin(s, DMC_KERNEL_ANCHORS);
  if (precision == DMC_FP64) {
    if (lay.anchor_bits > 0)
      hipLaunchKernelGGL(k_anchor_minmax<double>, dim3(AN_CHUNKS, 3, nw), dim3(kBlock), 0, s,
                         (const double*)frames, m.n, T, m.anchors, m.nc, part);
    hipLaunchKernelGGL(k_anchor_pack<double>, dim3(pk, 3, nw), dim3(kBlock), 0, s,
                       (const double*)frames, m.n, T, m.anchors, m.nc, lay.anchor_bits, part,
                       records, rec_bytes, lay);
  } else {
    if (lay.anchor_bits > 0)
      hipLaunchKernelGGL(k_anchor_minmax<float>, dim3(AN_CHUNKS, 3, nw), dim3(kBlock), 0, s,
                         (const float*)frames, m.n, T, m.anchors, m.nc, part);
    hipLaunchKernelGGL(k_anchor_pack<float>, dim3(pk, 3, nw), dim3(kBlock), 0, s,
                       (const float*)frames, m.n, T, m.anchors, m.nc, lay.anchor_bits, part,
                       records, rec_bytes, lay);
  }
  prof::end(s, DMC_KERNEL_ANCHORS);
}

void launch_dict_code(hipStream_t s, const double* u_canon, int32_t nw, const RecordLayout& lay,
                      uint8_t* records, size_t rec_bytes, double* u_tilde) {
  // differences chain the windows in one block; otherwise one block each
  const int per = lay.dict_mode == 1 ? nw : 1;
  const dim3 grid(lay.dict_mode == 1 ? 1 : nw);
  if (lay.precision == DMC_FP64)
    hipLaunchKernelGGL(k_dict_code<double>, grid, dim3(kBlock), 0, s, u_canon, nw, per, lay,
                       records, rec_bytes, u_tilde);
  else
    hipLaunchKernelGGL(k_dict_code<float>, grid, dim3(kBlock), 0, s, u_canon, nw, per, lay,
                       records, rec_bytes, u_tilde);
}

void launch_zero_tail(hipStream_t s, uint8_t* records, int32_t nw, size_t rec_bytes) {
  const int chunks = std::max(1, std::min(256, (int)((rec_bytes / 8 + 4 * kBlock - 1) / (4 * kBlock))));
  hipLaunchKernelGGL(k_zero_tail, dim3(chunks, nw), dim3(kBlock), 0, s, records, rec_bytes);
}

void launch_write_headers(hipStream_t s, uint8_t* records, int32_t nw, size_t rec_bytes,
                          const RecordLayout& l) {
  if (nw > 0) hipLaunchKernelGGL(k_header, dim3(nw), dim3(64), 0, s, records, rec_bytes, l);
}

}  // namespace dmc
