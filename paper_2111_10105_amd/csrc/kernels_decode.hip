// Decoder kernels (Eq. 12): dequantisation and back-projection of every
// window, the right-hand side of the normal equations, conjugate gradients on
// (L^T L + I_N^T I_N) X = L^T B + I_N^T A_N for all columns at once, and the
// final transpose to frames.
//
// Decoder vectors are float64 and vertex-major: row i holds the 3F values of
// vertex i, column j = 3 t + c for global frame t and coordinate c, so every
// sparse row gather is one contiguous read of a neighbour's row.
#include <algorithm>

#include "dmc_internal.h"
#include "wave_ops.h"

namespace dmc {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int CG_RB = 32;  // rows per CG block

__device__ inline double dequant(uint32_t code, double lo, double hi, int bits) {
#pragma clang fp contract(off)
  const double levels = (double)((1u << bits) - 1u);
  const double step = (hi - lo) / levels;
  return lo + (double)code * step;
}

// The record of window w.  The layout is returned by value: taking the
// address of a member of the by-value kernel argument would place the whole
// argument in scratch memory and turn every field read into a scratch load.
__device__ inline void window_of(const SeqLayout& sl, const uint8_t* records, int w,
                                 const uint8_t*& rec, int& T, int& k, int& t0,
                                 RecordLayout& lay) {
  if (w < sl.nw_full) {
    rec = records + (size_t)w * sl.rec_bytes_full;
    T = sl.T;
    k = sl.full.k;
    t0 = w * sl.T;
    lay = sl.full;
  } else {
    rec = records + (size_t)sl.nw_full * sl.rec_bytes_full;
    T = sl.T_tail;
    k = sl.tail.k;
    t0 = sl.nw_full * sl.T;
    lay = sl.tail;
  }
}

// The dequantised dictionary of window w in the decoder's u_tilde
// [window][3][T][k] (the short last window after the full ones).
__device__ inline const double* dict_of(const SeqLayout& sl, const double* ut, int w) {
  return ut + (size_t)(w < sl.nw_full ? w : sl.nw_full) * 3 * sl.T * sl.full.k;
}

// Dictionary decoder: for windows [w0, w1) of one group in order (block =
// group; wave v takes columns q = v, v + 4, ... of a window, lane = frame),
// the dequantised dictionary from the column table and packed segments:
// values, or the difference from the previous window's column.
template <typename Real>
__global__ void __launch_bounds__(kBlock)
k_dict_decode(const uint8_t* __restrict__ records, size_t rec_bytes, RecordLayout l, int nw,
              int per_block, double* __restrict__ ut) {
  const int T = l.T, k = l.k, nq = 3 * k;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int w0 = blockIdx.x * per_block, w1 = min(nw, w0 + per_block);
  for (int w = w0; w < w1; ++w) {
    const uint8_t* rec = records + (size_t)w * rec_bytes;
    const SegEntry* tab = (const SegEntry*)(rec + l.off_dtab);
    const uint32_t* var = (const uint32_t*)(rec + l.off_var);
    double* Ut = ut + (size_t)w * 3 * T * k;
    const double* Up = Ut - (size_t)3 * T * k;  // previous window (difference columns only)
    for (int q = wave; q < nq; q += kBlock / 64) {
      const int c = q / k, j = q % k, t = lane;
      if (t >= T) continue;
      const SegEntry e = tab[q];
      const uint32_t* seg = var + e.word_off;
      const uint32_t bits = e.bits_mode & 0xffu, mode = (e.bits_mode >> 8) & 0xffu;
      const size_t at = ((size_t)c * T + t) * k + j;
      double v;
      if (l.dict_bits == 0)
        v = (double)((const Real*)seg)[t];
      else
        v = bits ? dequant(get_code(seg, (uint32_t)t, bits), (double)e.lo, (double)e.hi, (int)bits)
                 : (double)e.lo;
      Ut[at] = mode ? Up[at] + v : v;
    }
    __syncthreads();
  }
}

// Dense anchor values Ahat[slot][j] for every column j of the sequence.
template <typename Real>
__global__ void k_anchor_values(const uint8_t* __restrict__ records, SeqLayout sl, int nc,
                                int ncols, double* __restrict__ Ah) {
  const size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= (size_t)nc * ncols) return;
  const int s = (int)(e / ncols), j = (int)(e % ncols);
  const int tg = j / 3, c = j % 3;
  int w = tg / sl.T;
  if (w > sl.nw_full) w = sl.nw_full;
  const uint8_t* rec;
  int T, k, t0;
  RecordLayout lay;
  window_of(sl, records, w, rec, T, k, t0, lay);
  const int t = tg - t0;
  const uint32_t idx = (uint32_t)t * nc + s;
  const uint32_t* seg = (const uint32_t*)(rec + lay.off_anchors + (size_t)c * lay.anchor_seg);
  double v;
  if (lay.anchor_bits > 0) {
    const float* rg = (const float*)(rec + lay.off_arange) + 2 * c;
    v = dequant(get_code(seg, idx, (uint32_t)lay.anchor_bits), (double)rg[0], (double)rg[1],
                lay.anchor_bits);
  } else {
    v = (double)((const Real*)seg)[idx];
  }
  Ah[e] = v;
}

// ---- right-hand side ------------------------------------------------------------
// k_rhs: a block takes CG_RB consecutive rows and SP_CW columns (SP_CPL per
// lane, 64 apart).  Row blocks go to the XCDs
// in contiguous runs: the x extent is padded to a multiple of the XCD count
// and block x takes row block (x mod 8) per + x / 8, so each XCD walks its
// own stretch of rows in order and finds the ring members' rows (a few
// positions away in the elimination order) in its L2.  The block's pattern
// (row offsets, column positions, values or weights) is staged in LDS first,
// so a wavefront's row loads wait on no index load of their own; each row's
// products go to four partial sums by entry index mod 4, added as
// (s0 + s1) + (s2 + s3).
constexpr int SP_CPL = 4, SP_CW = 64 * SP_CPL;
constexpr int SP_PAT = 1024;  // pattern entries staged per block (beyond: read from memory)

__device__ inline int xcd_row_block(int nrbp) {
  const int per = nrbp / kXcds;
  return (int)(blockIdx.x % kXcds) * per + (int)(blockIdx.x / kXcds);
}

// rows r0..r0+nr of the pattern into spr / scol / sval (sval[e] = wt(e))
template <typename Wt>
__device__ inline void stage_pattern(const int32_t* __restrict__ rowptr,
                                     const int32_t* __restrict__ col, int r0, int nr, int* spr,
                                     int* scol, double* sval, int& base, Wt wt) {
  for (int e = threadIdx.x; e <= nr; e += kBlock) spr[e] = rowptr[r0 + e];
  __syncthreads();
  base = spr[0];
  const int cnt = min(spr[nr] - base, SP_PAT);
  for (int e = threadIdx.x; e < cnt; e += kBlock) {
    const int c = col[base + e];
    scol[e] = c;
    sval[e] = wt(base + e, c);
  }
  __syncthreads();
}

// sum over row entries e0..e1 of wt(e) v[col(e)] for the lane's SP_CPL columns
template <typename Col, typename Wt>
__device__ inline void row_products(int e0, int e1, int ncols, const double* const (&vj)[SP_CPL],
                                    Col colof, Wt wtof, double (&out)[SP_CPL]) {
  double a[4][SP_CPL];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int u = 0; u < SP_CPL; ++u) a[q][u] = 0.0;
  int e = e0;
  for (; e + 4 <= e1; e += 4) {
    int c[4];
    double wq[4], xv[4][SP_CPL];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      c[q] = colof(e + q);
      wq[q] = wtof(e + q);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int u = 0; u < SP_CPL; ++u) xv[q][u] = vj[u][(size_t)c[q] * ncols];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int u = 0; u < SP_CPL; ++u) a[q][u] = fma(wq[q], xv[q][u], a[q][u]);
  }
  for (; e < e1; ++e) {
    const int c = colof(e);
    const double wv = wtof(e);
#pragma unroll
    for (int u = 0; u < SP_CPL; ++u) a[0][u] = fma(wv, vj[u][(size_t)c * ncols], a[0][u]);
  }
#pragma unroll
  for (int u = 0; u < SP_CPL; ++u) out[u] = (a[0][u] + a[1][u]) + (a[2][u] + a[3][u]);
}

// the block's per-column partial sums (wavefront order) into part[rb][j]
__device__ inline void block_column_partials(double (&v)[SP_CPL], double (*sh)[SP_CW], int ncols,
                                             int rb, double* __restrict__ part) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int u = 0; u < SP_CPL; ++u) sh[wv][lane + 64 * u] = v[u];
  __syncthreads();
  const int j = blockIdx.y * SP_CW + threadIdx.x;
  if (threadIdx.x < SP_CW && j < ncols) {
    double t = sh[0][threadIdx.x];
#pragma unroll
    for (int w = 1; w < kBlock / 64; ++w) t += sh[w][threadIdx.x];
    part[(size_t)rb * ncols + j] = t;
  }
}

// b = L^T B0 + I_N^T Ahat (the anchor term only when Ah is given), rows by
// position:
//   uniform:       (L^T u)_i = u_i - sum_{j in ring(i)} u_j / d_j
//   combinatorial: (L^T u)_i = d_i u_i - sum_{j in ring(i)} u_j
// (the ring weight is staged as 1 / d_j, or as 1 for the combinatorial
// form).  With bb given, also the block's partial b.b per column, the first
// half of the CG partials.
__global__ void __launch_bounds__(kBlock)
k_rhs(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
      const double* __restrict__ w, int uniform, const int32_t* __restrict__ slot, int n,
      int ncols, int nrbp, const double* __restrict__ B0, const double* __restrict__ Ah,
      double* __restrict__ b, double* __restrict__ bb) {
  constexpr int NW = kBlock / 64;
  __shared__ double sh[NW][SP_CW];
  __shared__ int spr[CG_RB + 1];
  __shared__ int scol[SP_PAT];
  __shared__ double sval[SP_PAT];
  const int rb = xcd_row_block(nrbp);
  const int r0 = rb * CG_RB;
  if (r0 >= n) return;  // padding block
  const int r1 = min(n, r0 + CG_RB);
  int base;
  stage_pattern(rowptr, col, r0, r1 - r0, spr, scol, sval, base,
                [&](int, int c) { return uniform ? w[c] : 1.0; });
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  int j[SP_CPL];
  bool jv[SP_CPL];
  const double* Bj[SP_CPL];
#pragma unroll
  for (int u = 0; u < SP_CPL; ++u) {
    j[u] = blockIdx.y * SP_CW + lane + 64 * u;
    jv[u] = j[u] < ncols;
    Bj[u] = B0 + (jv[u] ? j[u] : 0);
  }
  auto colof = [&](int e) { return e - base < SP_PAT ? scol[e - base] : col[e]; };
  auto wtof = [&](int e) {
    return e - base < SP_PAT ? sval[e - base] : (uniform ? w[col[e]] : 1.0);
  };
  double b2[SP_CPL];
#pragma unroll
  for (int u = 0; u < SP_CPL; ++u) b2[u] = 0.0;
  for (int i = r0 + wv; i < r1; i += NW) {
    double s[SP_CPL], ui[SP_CPL];
#pragma unroll
    for (int u = 0; u < SP_CPL; ++u) ui[u] = Bj[u][(size_t)i * ncols];
    row_products(spr[i - r0], spr[i - r0 + 1], ncols, Bj, colof, wtof, s);
    const double wi = w[i];
    const int sl = slot[i];
#pragma unroll
    for (int u = 0; u < SP_CPL; ++u) {
      double out = uniform ? ui[u] - s[u] : wi * ui[u] - s[u];
      if (Ah && sl >= 0 && jv[u]) out += Ah[(size_t)sl * ncols + j[u]];
      if (jv[u]) b[(size_t)i * ncols + j[u]] = out;
      b2[u] = fma(out, out, b2[u]);
    }
  }
  if (!bb) return;  // uniform over the block
  block_column_partials(b2, sh, ncols, rb, bb);
}

// ---- conjugate gradients ----------------------------------------------------

// x = 0 (only with zero_x: the first update writes x = alpha p), r = b (b may
// be r itself: the right-hand side is built in place), p = M^-1 r for the
// diagonal preconditioners (the Cholesky one sets p from its solve); partial
// b.b and r.z per column.
__global__ void __launch_bounds__(kBlock)
k_cg_init(const double* b, const double* __restrict__ dinv, int precond, int zero_x, int n,
          int ncols, double* __restrict__ x, double* r, double* __restrict__ p,
          double* __restrict__ part) {
  const int j = blockIdx.y * kBlock + threadIdx.x;
  if (j >= ncols) return;
  const int r0 = blockIdx.x * CG_RB, r1 = min(n, r0 + CG_RB);
  const bool copy_r = r != b;
  const bool set_p = precond != DMC_PRECOND_CHOLESKY;
  double bb = 0.0, rz = 0.0;
  for (int i = r0; i < r1; ++i) {
    const size_t e = (size_t)i * ncols + j;
    const double bv = b[e];
    const double z = precond == DMC_PRECOND_JACOBI ? dinv[i] * bv : bv;
    if (zero_x) x[e] = 0.0;
    if (copy_r) r[e] = bv;
    if (set_p) p[e] = z;
    bb += bv * bv;
    rz += bv * z;
  }
  const size_t nrb = gridDim.x;
  part[(size_t)blockIdx.x * ncols + j] = bb;
  part[(nrb + blockIdx.x) * ncols + j] = rz;
}

// Column sums of the per-block partials part[h][q][j] (h = 0, 1 selects the
// first or second half) by a block of 16 columns x 16 groups: group g adds the
// partials q = g, g + 16, ... into four independent sums (several loads in
// flight), and the sums and then the sixteen group sums are combined in a
// fixed order, so the result does not depend on scheduling.
constexpr int RED_COLS = 16, RED_GROUPS = kBlock / RED_COLS;

__device__ inline double column_sum(const double* __restrict__ part, int nrb, int ncols, int half,
                                    int j, double* sh) {
  const int g = threadIdx.x / RED_COLS, lc = threadIdx.x % RED_COLS;
  double acc = 0.0;
  if (j < ncols) {
    const double* pj = part + (size_t)half * nrb * ncols + j;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int q = g;
    // unrolled so that four rounds' loads are in flight together (the
    // accumulators and their order are unchanged)
#pragma unroll 4
    for (; q + 3 * RED_GROUPS < nrb; q += 4 * RED_GROUPS) {
      a0 += pj[(size_t)q * ncols];
      a1 += pj[(size_t)(q + RED_GROUPS) * ncols];
      a2 += pj[(size_t)(q + 2 * RED_GROUPS) * ncols];
      a3 += pj[(size_t)(q + 3 * RED_GROUPS) * ncols];
    }
    for (; q < nrb; q += RED_GROUPS) a0 += pj[(size_t)q * ncols];
    acc = (a0 + a1) + (a2 + a3);
  }
  sh[g * RED_COLS + lc] = acc;
  __syncthreads();
  double tot = 0.0;
  for (int h = 0; h < RED_GROUPS; ++h) tot += sh[h * RED_COLS + lc];
  __syncthreads();
  return tot;
}

__global__ void __launch_bounds__(kBlock)
k_cg_init_reduce(const double* __restrict__ part, int nrb, int ncols,
                 double* __restrict__ bnorm2, double* __restrict__ rz,
                 int32_t* __restrict__ done, double* __restrict__ resid) {
  // blockIdx.y = 0: the b.b half (and the flags that follow from it);
  // blockIdx.y = 1: the r.z half, in parallel
  __shared__ double sh[kBlock];
  const int j = blockIdx.x * RED_COLS + threadIdx.x % RED_COLS;
  const int half = blockIdx.y;
  const double v = column_sum(part, nrb, ncols, half, j, sh);
  if (j >= ncols || threadIdx.x >= RED_COLS) return;
  if (half == 1) {
    rz[j] = v;
    return;
  }
  bnorm2[j] = v;
  done[j] = v == 0.0 ? 1 : 0;
  resid[j] = v == 0.0 ? 0.0 : 1.0;
}

// q = M p (CSR of L^T L + I_N^T I_N, by position), partial p.q per column.  A block
// takes CG_RB rows and 64 columns (one per lane), row blocks in XCD runs as
// in k_rhs (the rows of a row's two rings stay in its XCD's L2); its four
// wavefronts take
// every fourth row, so each lane has a short chain of rows, and their p.q
// partials are added in wavefront order (deterministic).  The row's pattern
// and values are the same for the whole wavefront (scalar loads).
constexpr int SP_COLS = 64;
constexpr int SP_ROW = 20;  // gathers of a row issued together (M's rows: 19 at valence 6)
static_assert(SP_ROW <= kMatPad, "a row's first SP_ROW entries lie inside the padded arrays");

__global__ void __launch_bounds__(kBlock)
k_cg_spmm(const int32_t* __restrict__ mrow, const int32_t* __restrict__ mcol,
          const double* __restrict__ mval, int n, int ncols, const double* __restrict__ p,
          double* __restrict__ q, double* __restrict__ part) {
  constexpr int NW = kBlock / 64;
  __shared__ double sh[NW][SP_COLS];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int j = blockIdx.y * SP_COLS + lane;
  const bool jv = j < ncols;
  const double* pj = p + (jv ? j : 0);
  const int rb = xcd_row_block(gridDim.x);
  const int r0 = rb * CG_RB, r1 = min(n, r0 + CG_RB);
  if (r0 >= n) return;  // padding block
  double pq = 0.0;
  for (int i = r0 + wv; i < r1; i += NW) {
    const int e0 = mrow[i], e1 = mrow[i + 1], len = e1 - e0, full = len & ~3;
    // the row's first SP_ROW gathers are issued before any product; entries
    // in groups of four go to a[e mod 4], the remainder to a[0] (a chained
    // four-way sum); indices and weights are read without bounds tests (the
    // arrays carry kMatPad entries past their end)
    int cx[SP_ROW];
    double wx[SP_ROW], x[SP_ROW];
#pragma unroll
    for (int h = 0; h < SP_ROW; ++h) {
      cx[h] = mcol[e0 + h];
      wx[h] = mval[e0 + h];
    }
#pragma unroll
    for (int h = 0; h < SP_ROW; ++h) x[h] = h < len ? pj[(size_t)cx[h] * ncols] : 0.0;
    double a[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int h = 0; h < SP_ROW; ++h)
      if (h < len) a[h < full ? (h & 3) : 0] = fma(wx[h], x[h], a[h < full ? (h & 3) : 0]);
    for (int h = SP_ROW; h < len; ++h) {  // rows longer than SP_ROW
      const int q = h < full ? (h & 3) : 0;
      a[q] = fma(mval[e0 + h], pj[(size_t)mcol[e0 + h] * ncols], a[q]);
    }
    const double acc = (a[0] + a[1]) + (a[2] + a[3]);
    if (jv) q[(size_t)i * ncols + j] = acc;
    pq = fma(pj[(size_t)i * ncols], acc, pq);
  }
  sh[wv][lane] = pq;
  __syncthreads();
  if (threadIdx.x < SP_COLS && jv) {
    double v = sh[0][lane];
#pragma unroll
    for (int u = 1; u < NW; ++u) v += sh[u][lane];
    part[(size_t)rb * ncols + j] = v;
  }
}

// Residual of a start x0: partial (b - M x0).(b - M x0) per column into the
// first half of `part`; with write_r, r = b - M x0 is also written in place of
// b (each element is read and written by one thread).  Tiled as k_cg_spmm
// (row blocks in XCD runs, a wavefront's rows in a chain, the row's pattern
// in scalar registers), with CPL adjacent columns per lane: CPL = 2 (an even
// column count) reads each ring member's pair with one 16-byte load, which
// halves the load instructions per byte and the pattern loads per column.
// Each element's products are summed by entry index mod 4 as in k_cg_spmm.
constexpr int RS_ROW = 20;  // gathers of a row issued together (M's rows: 19 at valence 6)
static_assert(RS_ROW <= kMatPad, "a row's first RS_ROW entries lie inside the padded arrays");

template <int CPL>
__global__ void __launch_bounds__(kBlock)
k_cg_residual(const int32_t* __restrict__ mrow, const int32_t* __restrict__ mcol,
              const double* __restrict__ mval, int n, int ncols, const double* __restrict__ x,
              double* b, int write_r, double* __restrict__ part) {
  typedef double dv __attribute__((ext_vector_type(CPL)));
  constexpr int NW = kBlock / 64, BW = 64 * CPL;
  __shared__ double sh[NW][BW];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int j = blockIdx.y * BW + CPL * lane;
  const bool jv = j < ncols;  // CPL divides ncols
  const double* xj = x + (jv ? j : 0);
  const int rb = xcd_row_block(gridDim.x);
  const int r0 = rb * CG_RB, r1 = min(n, r0 + CG_RB);
  if (r0 >= n) return;  // padding block
  auto ld = [&](int c) { return *(const dv*)(xj + (size_t)c * ncols); };
  dv rr = {};
  for (int i = r0 + wv; i < r1; i += NW) {
    const int e0 = mrow[i], e1 = mrow[i + 1], len = e1 - e0, full = len & ~3;
    // the row's first RS_ROW gathers and its b value are all issued before
    // any product (the entries in groups of four go to a[e mod 4], the
    // remainder to a[0], the order of a chained four-way sum)
    const size_t at = (size_t)i * ncols + (jv ? j : 0);
    const dv bv = *(const dv*)(b + at);
    // indices and weights read without bounds tests (the arrays carry
    // kMatPad entries past their end)
    int cx[RS_ROW];
    double wx[RS_ROW];
#pragma unroll
    for (int h = 0; h < RS_ROW; ++h) {
      cx[h] = mcol[e0 + h];
      wx[h] = mval[e0 + h];
    }
    dv x[RS_ROW];
#pragma unroll
    for (int h = 0; h < RS_ROW; ++h) x[h] = h < len ? ld(cx[h]) : dv{};
    dv a[4] = {{}, {}, {}, {}};
#pragma unroll
    for (int h = 0; h < RS_ROW; ++h) {
      if (h < len) {
        const int q = h < full ? (h & 3) : 0;
        const double wt = wx[h];
#pragma unroll
        for (int u = 0; u < CPL; ++u) a[q][u] = fma(wt, x[h][u], a[q][u]);
      }
    }
    for (int h = RS_ROW; h < len; ++h) {  // rows longer than RS_ROW
      const int q = h < full ? (h & 3) : 0;
      const dv x0 = ld(mcol[e0 + h]);
#pragma unroll
      for (int u = 0; u < CPL; ++u) a[q][u] = fma(mval[e0 + h], x0[u], a[q][u]);
    }
    const dv a0 = a[0], a1 = a[1], a2 = a[2], a3 = a[3];
    if (jv) {
      dv rv = bv;
#pragma unroll
      for (int u = 0; u < CPL; ++u) {
        rv[u] -= (a0[u] + a1[u]) + (a2[u] + a3[u]);
        rr[u] = fma(rv[u], rv[u], rr[u]);
      }
      if (write_r) *(dv*)(b + at) = rv;
    }
  }
#pragma unroll
  for (int u = 0; u < CPL; ++u) sh[wv][CPL * lane + u] = rr[u];
  __syncthreads();
  const int jj = blockIdx.y * BW + threadIdx.x;
  if (threadIdx.x < BW && jj < ncols) {
    double v = sh[0][threadIdx.x];
#pragma unroll
    for (int u = 1; u < NW; ++u) v += sh[u][threadIdx.x];
    part[(size_t)rb * ncols + jj] = v;
  }
}

// rz[j] = column sum of the second half of the partials (r.z)
__global__ void __launch_bounds__(kBlock)
k_cg_rz_reduce(const double* __restrict__ part, int nrb, int ncols, double* __restrict__ rz) {
  __shared__ double sh[kBlock];
  const int j = blockIdx.x * RED_COLS + threadIdx.x % RED_COLS;
  const double v = column_sum(part, nrb, ncols, 1, j, sh);
  if (j >= ncols || threadIdx.x >= RED_COLS) return;
  rz[j] = v;
}

__global__ void __launch_bounds__(kBlock)
k_cg_alpha(const double* __restrict__ part, int nrb, int ncols,
           const double* __restrict__ rz, const int32_t* __restrict__ done,
           double* __restrict__ alpha) {
  __shared__ double sh[kBlock];
  const int j = blockIdx.x * RED_COLS + threadIdx.x % RED_COLS;
  const double pq = column_sum(part, nrb, ncols, 0, j, sh);
  if (j >= ncols || threadIdx.x >= RED_COLS) return;
  alpha[j] = (done[j] || pq == 0.0) ? 0.0 : rz[j] / pq;
}

__global__ void __launch_bounds__(kBlock)
k_cg_update(int n, int ncols, const double* __restrict__ alpha, const double* __restrict__ dinv,
            int precond, int first, double* __restrict__ x, double* __restrict__ r,
            const double* __restrict__ p, const double* __restrict__ q, double* __restrict__ part) {
  // 64 columns per block, its four wavefronts on every fourth row; the
  // partials are added in wavefront order
  constexpr int NW = kBlock / 64;
  __shared__ double sh[2][NW][SP_COLS];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int j = blockIdx.y * SP_COLS + lane;
  const bool jv = j < ncols;
  const int r0 = blockIdx.x * CG_RB, r1 = jv ? min(n, r0 + CG_RB) : r0;
  const double a = jv ? alpha[j] : 0.0;
  double rr = 0.0, rz = 0.0;
  for (int i = r0 + wv; i < r1; i += NW) {
    const size_t e = (size_t)i * ncols + j;
    // from x = 0 the first update is alpha p (fma(a, p, 0) = a p exactly)
    x[e] = first ? a * p[e] : fma(a, p[e], x[e]);
    const double rv = fma(-a, q[e], r[e]);
    r[e] = rv;
    const double z = precond == DMC_PRECOND_JACOBI ? dinv[i] * rv : rv;
    rr = fma(rv, rv, rr);
    rz = fma(rv, z, rz);
  }
  sh[0][wv][lane] = rr;
  sh[1][wv][lane] = rz;
  __syncthreads();
  if (threadIdx.x >= SP_COLS || !jv) return;
  double vrr = sh[0][0][lane], vrz = sh[1][0][lane];
#pragma unroll
  for (int u = 1; u < NW; ++u) {
    vrr += sh[0][u][lane];
    vrz += sh[1][u][lane];
  }
  const size_t nrb = gridDim.x;
  part[(size_t)blockIdx.x * ncols + j] = vrr;
  // with the Cholesky preconditioner r.z comes from k_cg_dot after the solve
  if (precond != DMC_PRECOND_CHOLESKY) part[(nrb + blockIdx.x) * ncols + j] = vrz;
}

// partial r.z per column into the second half of `part`; with p given, also
// p = z (the first search direction)
__global__ void __launch_bounds__(kBlock)
k_cg_dot(int n, int ncols, const double* __restrict__ r, const double* __restrict__ z,
         double* __restrict__ p, double* __restrict__ part) {
  // 64 columns per block, its four wavefronts on every fourth row; the
  // partials are added in wavefront order
  constexpr int NW = kBlock / 64;
  __shared__ double sh[NW][SP_COLS];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int j = blockIdx.y * SP_COLS + lane;
  const bool jv = j < ncols;
  const int r0 = blockIdx.x * CG_RB, r1 = jv ? min(n, r0 + CG_RB) : r0;
  double rz = 0.0;
  for (int i = r0 + wv; i < r1; i += NW) {
    const size_t e = (size_t)i * ncols + j;
    const double zv = z[e];
    rz = fma(r[e], zv, rz);
    if (p) p[e] = zv;
  }
  sh[wv][lane] = rz;
  __syncthreads();
  if (threadIdx.x >= SP_COLS || !jv) return;
  double v = sh[0][lane];
#pragma unroll
  for (int u = 1; u < NW; ++u) v += sh[u][lane];
  part[((size_t)gridDim.x + blockIdx.x) * ncols + j] = v;
}

// relative residual per column from the r.r partials; marks converged columns
__global__ void __launch_bounds__(kBlock)
k_cg_resid(const double* __restrict__ part, int nrb, int ncols,
           const double* __restrict__ bnorm2, int32_t* __restrict__ done,
           double* __restrict__ resid, double tol) {
  __shared__ double sh[kBlock];
  const int j = blockIdx.x * RED_COLS + threadIdx.x % RED_COLS;
  const double rr = column_sum(part, nrb, ncols, 0, j, sh);
  if (j >= ncols || threadIdx.x >= RED_COLS) return;
  if (done[j]) return;
  const double res = bnorm2[j] > 0.0 ? sqrt(rr / bnorm2[j]) : 0.0;
  resid[j] = res;
  if (res <= tol) done[j] = 2;  // converged in this iteration
}

// beta = (r.z)_new / (r.z)_old from the r.z partials (zero for converged columns)
__global__ void __launch_bounds__(kBlock)
k_cg_beta(const double* __restrict__ part, int nrb, int ncols,
          double* __restrict__ rz, int32_t* __restrict__ done,
          double* __restrict__ beta) {
  __shared__ double sh[kBlock];
  const int j = blockIdx.x * RED_COLS + threadIdx.x % RED_COLS;
  const double z = column_sum(part, nrb, ncols, 1, j, sh);
  if (j >= ncols || threadIdx.x >= RED_COLS) return;
  if (done[j]) {
    done[j] = 1;
    beta[j] = 0.0;
    return;
  }
  beta[j] = rz[j] != 0.0 ? z / rz[j] : 0.0;
  rz[j] = z;
}

__global__ void __launch_bounds__(kBlock)
k_cg_pupdate(int n, int ncols, const double* __restrict__ beta, const double* __restrict__ dinv,
             int precond, const double* __restrict__ r, const double* __restrict__ zarr,
             double* __restrict__ p) {
  const int j = blockIdx.y * kBlock + threadIdx.x;
  if (j >= ncols) return;
  const int r0 = blockIdx.x * CG_RB, r1 = min(n, r0 + CG_RB);
  const double bt = beta[j];
  for (int i = r0; i < r1; ++i) {
    const size_t e = (size_t)i * ncols + j;
    const double z = precond == DMC_PRECOND_CHOLESKY ? zarr[e]
                     : precond == DMC_PRECOND_JACOBI ? dinv[i] * r[e]
                                                     : r[e];
    p[e] = fma(bt, p[e], z);
  }
}

// X [n][3F] (row pos(i) for vertex i) -> frames [F][n][3].  Block = TF_V
// vertices x TF_T frames: each vertex's 3 TF_T values are one contiguous run
// of X (read with TF_U loads in flight per thread), held in LDS in the frames'
// type, and written frame by frame as runs of 3 TF_V values.  Long write runs
// pay more than long read runs: at icosphere 7 (F = 512) 128 x 16 took 0.61
// ms, 64 x 32 0.67, 32 x 64 0.73, 16 x 128 0.85 (256 x 8 as 128 x 16).
constexpr int TF_V = 128, TF_T = 16, TF_U = 8;

template <typename Real>
__global__ void __launch_bounds__(kBlock)
k_to_frames(const double* __restrict__ X, const int32_t* __restrict__ pos, int n, int F,
            Real* __restrict__ out) {
  constexpr int RW = 3 * TF_T, LD = RW + 1;
  __shared__ Real tile[TF_V * LD];
  __shared__ int prow[TF_V];
  const int i0 = blockIdx.x * TF_V, t0 = blockIdx.y * TF_T;
  const int ncols = 3 * F;
  const int nv = min(TF_V, n - i0), nt = min(TF_T, F - t0);
  if (threadIdx.x < TF_V) prow[threadIdx.x] = threadIdx.x < nv ? pos[i0 + threadIdx.x] : 0;
  __syncthreads();
  // the tile is whole rounds of TF_U loads per thread, and items beyond the
  // block's vertices or frames read an in-range value that is never written
  // out: no load sits behind a branch, so all TF_U are in flight at once
  static_assert(TF_V * RW % (TF_U * kBlock) == 0, "whole rounds");
  for (int e0 = threadIdx.x; e0 < TF_V * RW; e0 += TF_U * kBlock) {
    double v[TF_U];
#pragma unroll
    for (int u = 0; u < TF_U; ++u) {
      const int e = e0 + u * kBlock;
      const int vv = min(e / RW, nv - 1), j = min(e % RW, 3 * nt - 1);
      v[u] = X[(size_t)prow[vv] * ncols + 3 * t0 + j];
    }
#pragma unroll
    for (int u = 0; u < TF_U; ++u) {
      const int e = e0 + u * kBlock;
      tile[(e / RW) * LD + e % RW] = (Real)v[u];
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < TF_T * 3 * TF_V; e += kBlock) {
    const int t = e / (3 * TF_V), vc = e % (3 * TF_V);
    const int vv = vc / 3, c = vc % 3;
    if (t < nt && vv < nv) out[((size_t)(t0 + t) * n + i0 + vv) * 3 + c] = tile[vv * LD + 3 * t + c];
  }
}

// ---- temporal-subspace decode ------------------------------------------------
// Eq. (12) is linear in its right-hand side, and the right-hand side of window
// w and coordinate c is L^T Y^_wc^T U~_wc^T + I_N^T A^_wc.  So
//   X_wc = Z_wc U~_wc^T + G A^_wc,
// where Z_wc (n x k) solves the normal equations for the k columns L^T Y^_wc^T
// and G = (L^T L + I_N^T I_N)^{-1} I_N^T (n x nc) is the anchor response of
// the mesh, solved once.  The reduced system has 3k columns per window
// instead of 3T.  Column of coefficient r of coordinate c of window w:
// zoff(w) + c k_w + r.
__device__ inline int zoff(const SeqLayout& sl, int w) {
  return 3 * sl.full.k * (w < sl.nw_full ? w : sl.nw_full);
}

// vertices per block of k_coef_rows (at icosphere 7: 32 -> 0.37 ms, 64 -> 0.40,
// 16 -> 0.39; the smaller tile lets more blocks share a CU)
constexpr int CR_V = 32;
constexpr int CR_U = 8;   // codes in flight per thread

// Yd[pos(i)][zoff(w) + c k + r] = Y^_wc[r][i] (dequantised coefficients, one
// row per vertex in the decoder's row order).  The window's row table is
// staged in LDS first, so each code's load depends on no table load of its
// own; consecutive threads read consecutive vertices of a row.  A code is
// read as two words without a branch (the second is the first again when
// the code does not cross a word boundary; a constant row reads the record's
// first word and uses none of it), so all 2 CR_U words of a thread's codes
// are in flight at once; the value is that of get_code.
template <typename Real>
__global__ void __launch_bounds__(kBlock)
k_coef_rows(const uint8_t* __restrict__ records, SeqLayout sl, int n, int nz,
            const int32_t* __restrict__ pos, double* __restrict__ Yd) {
  __shared__ double tile[CR_V * 97];  // [v][c k + r], 3k <= 96
  __shared__ SegEntry tab[96];
  __shared__ int prow[CR_V];
  const int w = blockIdx.y;
  const uint8_t* rec;
  int T, k, t0;
  RecordLayout lay;
  window_of(sl, records, w, rec, T, k, t0, lay);
  const int i0 = blockIdx.x * CR_V;
  const int nv = min(CR_V, n - i0);
  const int ck = 3 * k;
  if (threadIdx.x < ck) tab[threadIdx.x] = ((const SegEntry*)(rec + lay.off_rtab))[threadIdx.x];
  if (threadIdx.x < CR_V) prow[threadIdx.x] = threadIdx.x < nv ? pos[i0 + threadIdx.x] : 0;
  __syncthreads();
  const uint32_t* var = (const uint32_t*)(rec + lay.off_var);
  const uint32_t* first = (const uint32_t*)rec;
  const int tot = ck * CR_V;
  for (int e0 = threadIdx.x; e0 < tot; e0 += CR_U * kBlock) {
    double y[CR_U];
    if (lay.coef_bits == 0) {
#pragma unroll
      for (int u = 0; u < CR_U; ++u) {
        const int e = e0 + u * kBlock;
        const int cr = e / CR_V, v = e % CR_V;
        y[u] = (e < tot && v < nv) ? (double)((const Real*)(var + tab[cr].word_off))[i0 + v] : 0.0;
      }
    } else {
      uint32_t wlo[CR_U], whi[CR_U];
#pragma unroll
      for (int u = 0; u < CR_U; ++u) {
        // out-of-range items read an in-range code and are dropped below
        const int e = e0 + u * kBlock;
        const int cr = min(e / CR_V, ck - 1), v = min(e % CR_V, nv - 1);
        const SegEntry se = tab[cr];
        const uint32_t bits = se.bits_mode & 0xffu;
        const uint64_t at = (uint64_t)(uint32_t)(i0 + v) * bits;
        const uint32_t sh = (uint32_t)(at & 31);
        const uint32_t* p = bits ? var + se.word_off + (uint32_t)(at >> 5) : first;
        wlo[u] = p[0];
        whi[u] = p[sh + bits > 32 ? 1 : 0];
      }
#pragma unroll
      for (int u = 0; u < CR_U; ++u) {
        const int e = e0 + u * kBlock;
        const int cr = e / CR_V, v = e % CR_V;
        y[u] = 0.0;
        if (e < tot && v < nv) {
          const SegEntry se = tab[cr];
          const uint32_t bits = se.bits_mode & 0xffu;
          const uint32_t sh = (uint32_t)(((uint64_t)(uint32_t)(i0 + v) * bits) & 31);
          const uint64_t word = (uint64_t)wlo[u] | ((uint64_t)whi[u] << 32);
          const uint32_t code = (uint32_t)(word >> sh) & ((1u << bits) - 1u);
          y[u] = bits ? dequant(code, (double)se.lo, (double)se.hi, (int)bits) : (double)se.lo;
        }
      }
    }
#pragma unroll
    for (int u = 0; u < CR_U; ++u) {
      const int e = e0 + u * kBlock;
      if (e < tot) tile[(e % CR_V) * 97 + e / CR_V] = y[u];
    }
  }
  __syncthreads();
  const int z0 = zoff(sl, w);
  for (int e = threadIdx.x; e < nv * ck; e += kBlock) {
    const int v = e / ck, cr = e % ck;
    Yd[(size_t)prow[v] * nz + z0 + cr] = tile[v * 97 + cr];
  }
}

// Right-hand side of the direct decode from the coefficient rows: Eq. (12)'s
// L^T B0 with B0 = Y^_wc^T U~_wc^T per window and coordinate equals
// (L^T Y^_wc^T) U~_wc^T, so the Laplacian runs on the 3k coefficient columns
// of a window instead of its 3T frame columns and the back-projected
// deltas are never stored:
//   b[pos(i)][3(t0+t)+c] = sum_r U~_c[t][r] (L^T Yd)[i][zoff(w) + c k + r]
//                          (+ A^[slot][j] at anchor rows)
// Block (CG row block of CG_RB rows, window w):
//  1. the block's rings in LDS, padded to RX_RING entries (weight 0 on the
//     row itself), so a thread issues the loads of two (row, column) items
//     at once without waiting on a loop bound; longer rings finish from
//     memory;
//  2. z = L^T Yd for the window's 3k columns into LDS (ring weights as in
//     k_rhs);
//  3. the expansion on the FP64 matrix cores: a wavefront takes a 16-frame
//     tile and a run of 16-row tiles (the dictionary operands of its frames
//     stay in registers), puts the three coordinates' results of 4 rows at
//     a time into its own LDS stage in b's column order, and writes them
//     out as contiguous runs.
// With bb given, the block's b.b partial per column (k_rhs's row blocks),
// summed in a fixed order.  KM: the largest k of the sequence (16 or 32).
constexpr int RX_RING = 8;

template <int KM>
__global__ void __launch_bounds__(kBlock)
k_rhs_expand(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
             const double* __restrict__ w, int uniform, const int32_t* __restrict__ slot, int n,
             int ncols, int nz, int nrbp, SeqLayout sl, const double* __restrict__ Yd,
             const double* __restrict__ ut, const double* __restrict__ Ah,
             double* __restrict__ b, double* __restrict__ bb) {
  constexpr int ZST = 3 * KM + 1;  // row stride of zs (odd: rows on different banks)
  constexpr int NW = kBlock / 64;
  __shared__ double zs[CG_RB * ZST];           // [v][c k + r]
  __shared__ double stage[NW][4 * 48];         // per wave: 4 rows x (16 frames x 3)
  __shared__ int rcol[CG_RB][RX_RING];
  __shared__ double rwt[CG_RB][RX_RING];
  __shared__ int rlen[CG_RB + 1];
  __shared__ int sslot[CG_RB];
  __shared__ double sq[CG_RB / 16][3][64];     // per row tile: column sums of b^2
  const int rb = xcd_row_block(nrbp);
  const int r0 = rb * CG_RB;
  if (r0 >= n) return;  // padding block
  const int nr = min(CG_RB, n - r0);
  const int win = blockIdx.y;
  const bool full = win < sl.nw_full;
  const int T = full ? sl.T : sl.T_tail, k = full ? sl.full.k : sl.tail.k;
  const int t0 = (full ? win : sl.nw_full) * sl.T;
  const int ck = 3 * k, z0 = zoff(sl, win);
  // 1. rings (rlen[v] = start of row v's entries; rows past n empty)
  for (int v = threadIdx.x; v <= CG_RB; v += kBlock) rlen[v] = rowptr[r0 + min(v, nr)];
  for (int v = threadIdx.x; v < CG_RB; v += kBlock) sslot[v] = v < nr ? slot[r0 + v] : -1;
  __syncthreads();
  for (int e = threadIdx.x; e < CG_RB * RX_RING; e += kBlock) {
    const int v = e / RX_RING, h = e % RX_RING;
    const int q = rlen[v] + h;
    const bool on = v < nr && q < rlen[v + 1];
    const int cj = on ? col[q] : min(r0 + v, n - 1);
    rcol[v][h] = cj;
    rwt[v][h] = on ? (uniform ? w[cj] : 1.0) : 0.0;
  }
  __syncthreads();
  // 2. z rows: item e = (row e / ck, column e % ck), two items per pass
  auto zitem = [&](int v, int cr, double (&x)[RX_RING + 1]) {
    const double* yc = Yd + z0 + cr;
#pragma unroll
    for (int h = 0; h < RX_RING; ++h) x[h] = yc[(size_t)rcol[v][h] * nz];
    x[RX_RING] = yc[(size_t)min(r0 + v, n - 1) * nz];
  };
  auto zfinish = [&](int v, int cr, const double (&x)[RX_RING + 1]) {
    double a[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int h = 0; h < RX_RING; ++h) a[h % 4] = fma(rwt[v][h], x[h], a[h % 4]);
    const double* yc = Yd + z0 + cr;
    for (int q = rlen[v] + RX_RING; q < rlen[v + 1]; ++q) {  // rings longer than RX_RING
      const int cj = col[q];
      a[0] = fma(uniform ? w[cj] : 1.0, yc[(size_t)cj * nz], a[0]);
    }
    const double s4 = (a[0] + a[1]) + (a[2] + a[3]);
    const double ui = x[RX_RING];
    return v < nr ? (uniform ? ui - s4 : w[r0 + v] * ui - s4) : 0.0;
  };
  const int nitem = CG_RB * ck;
  for (int e = threadIdx.x; e < nitem; e += 2 * kBlock) {
    const int e2 = e + kBlock;
    const int v1 = e / ck, c1 = e % ck;
    const int v2 = e2 < nitem ? e2 / ck : v1, c2 = e2 < nitem ? e2 % ck : c1;
    double x1[RX_RING + 1], x2[RX_RING + 1];
    zitem(v1, c1, x1);
    zitem(v2, c2, x2);
    zs[v1 * ZST + c1] = zfinish(v1, c1, x1);
    if (e2 < nitem) zs[v2 * ZST + c2] = zfinish(v2, c2, x2);
  }
  __syncthreads();
  // 3. expansion.  Item (tt, g): frames 16 tt.. and row tiles g rts ..; lane l
  // supplies A[l%16][l/16] = z[row][c k + 4 s + l/16] and B[l/16][l%16] =
  // U~_c[t][4 s + l/16]; component q of lane l is row 4 q + l/16, frame l%16
  const double* U = ut + (size_t)(full ? win : sl.nw_full) * 3 * sl.T * sl.full.k;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int l16 = lane & 15, lg = lane >> 4;
  const int nT16 = (T + 15) >> 4;
  constexpr int NRT = CG_RB / 16;
  const int groups = max(1, min(NW / nT16, NRT)), rts = NRT / groups;
  double* st = stage[wv];
  for (int it = wv; it < nT16 * groups; it += NW) {
    const int tt = it % nT16, g = it / nT16;
    const int t = 16 * tt + l16;
    const int nt = min(16, T - 16 * tt);  // frames of this tile
    double bu[3][KM / 4];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int s = 0; s < KM / 4; ++s) {
        const int r = 4 * s + lg;
        bu[c][s] = (t < T && r < k) ? U[((size_t)c * T + t) * k + r] : 0.0;
      }
    for (int rt = g * rts; rt < (g + 1) * rts; ++rt) {
      const double* zrow = zs + (16 * rt + l16) * ZST;
      d4 acc[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        acc[c] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < KM / 4; ++s) {
          const int r = 4 * s + lg;
          if (4 * s < k) {
            const double az = r < k ? zrow[c * k + r] : 0.0;
            acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(az, bu[c][s], acc[c], 0, 0, 0);
          }
        }
      }
      // anchor term and column sums of squares (lane: frame t, rows 4 q + lg)
      double sqs[3] = {0.0, 0.0, 0.0};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int v = 16 * rt + 4 * q + lg;
        const int sv = v < nr ? sslot[v] : -1;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          double val = acc[c][q];
          if (Ah && sv >= 0 && t < T) val += Ah[(size_t)sv * ncols + 3 * (t0 + t) + c];
          acc[c][q] = val;
          if (v < nr && t < T) sqs[c] = fma(val, val, sqs[c]);
        }
      }
      if (bb) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          // the tile's column sum over lanes l16, l16 + 16, l16 + 32, l16 + 48
          double x = sqs[c] + swap16_f64(sqs[c]);
          x += shfl_f64(x, lane ^ 32);
          if (lg == 0) sq[rt][c][t] = x;
        }
      }
      // rows 4 q + lg, four at a time (one q): stage in b's column order
      // (3 t + c), then contiguous runs of 3 nt values per row
#pragma unroll
      for (int q = 0; q < 4; ++q) {
#pragma unroll
        for (int c = 0; c < 3; ++c) st[lg * 48 + 3 * l16 + c] = acc[c][q];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        for (int e = lane; e < 4 * 48; e += 64) {
          const int vr = e / 48, cc = e % 48;
          // staged row vr is tile row 4 q + vr (lanes with l/16 = vr wrote it)
          const int v = 16 * rt + 4 * q + vr;
          if (v < nr && cc < 3 * nt)
            b[(size_t)(r0 + v) * ncols + 3 * (t0 + 16 * tt) + cc] = st[e];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
    }
  }
  if (!bb) return;  // uniform over the block
  __syncthreads();
  for (int e = threadIdx.x; e < 3 * T; e += kBlock) {
    const int t = e / 3, c = e % 3;
    bb[(size_t)rb * ncols + 3 * (t0 + t) + c] = sq[0][c][t] + sq[1][c][t];
  }
}

// right-hand sides of the anchor response: b[p][a] = 1 if the vertex at row
// position p is anchor a (slot by position)
__global__ void __launch_bounds__(kBlock)
k_anchor_unit_rhs(const int32_t* __restrict__ slot, int n, int nc, double* __restrict__ b) {
  const size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= (size_t)n * nc) return;
  const int i = (int)(e / nc), a = (int)(e % nc);
  b[e] = slot[i] == a ? 1.0 : 0.0;
}

constexpr int GR_ROWS = 512;  // rows per partial Gram block

// Partial Gram matrices b_g^T b_g of the groups g = 3 w + c of the reduced
// right-hand side b [n][nz] (the k columns of window w, coordinate c).  Block
// (g, chunk) adds rows chunk*GR_ROWS.. in order; part[g][chunk][k*k] (stride kk2).
__global__ void __launch_bounds__(kBlock)
k_group_gram(SeqLayout sl, int n, int nz, int kk2, const double* __restrict__ b,
             double* __restrict__ part) {
  __shared__ double rows[64 * 33];
  const int g = blockIdx.x, chunk = blockIdx.y;
  const int w = g / 3, c = g % 3;
  const int k = w < sl.nw_full ? sl.full.k : sl.tail.k;
  const int col0 = zoff(sl, w) + c * k;
  const int r0 = chunk * GR_ROWS, r1 = min(n, r0 + GR_ROWS);
  double acc[4] = {0.0, 0.0, 0.0, 0.0};  // entries threadIdx.x + q * kBlock (k*k <= 1024)
  // the next 64-row tile is loaded into registers (every load in flight)
  // while the current one is multiplied
  constexpr int PT = 64 * 32 / kBlock;  // tile elements per thread (k <= 32)
  double pre[PT];
  auto load = [&](int i0) {
    const int nv = min(64, r1 - i0);
#pragma unroll
    for (int u = 0; u < PT; ++u) {
      const int e = threadIdx.x + u * kBlock, v = e / k, r = e % k;
      pre[u] = (e < 64 * k && v < nv) ? b[(size_t)(i0 + v) * nz + col0 + r] : 0.0;
    }
  };
  if (r0 < r1) load(r0);
  for (int i0 = r0; i0 < r1; i0 += 64) {
    const int nv = min(64, r1 - i0);
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PT; ++u) {
      const int e = threadIdx.x + u * kBlock;
      if (e < 64 * k) rows[(e / k) * 33 + e % k] = pre[u];
    }
    __syncthreads();
    if (i0 + 64 < r1) load(i0 + 64);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = threadIdx.x + q * kBlock;
      if (e < k * k) {
        const int r = e / k, s = e % k;
        double a = acc[q];
        for (int v = 0; v < nv; ++v) a = fma(rows[v * 33 + r], rows[v * 33 + s], a);
        acc[q] = a;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int e = threadIdx.x + q * kBlock;
    if (e < k * k) part[((size_t)g * gridDim.y + chunk) * kk2 + e] = acc[q];
  }
}

// Reference norms of the reduced columns, so that the conjugate-gradient test
// on them bounds the residual of every frame's full system: frame t of group
// g = (w, c) has right-hand side B_t = sum_r b_r U~[t][r] + I_N^T A^_t and
// residual sum_r rho_r U~[t][r] + rho_G A^_t, with
//   ||B_t||^2 = u^T Gram u + 2 u . s + ||A^_t||^2   (u = U~[t], s_r = sum_a
//   b_r[anchor a] A^[a][t]),  ||rho_G A^_t|| <= g_resid ||A^_t||_1.
// With allowance_t = tol ||B_t|| - g_resid ||A^_t||_1, the test
// sum_r ||rho_r||^2 <= min_t allowance_t^2 (rows of U~ have norm <= 1) gives
// ||residual_t|| <= tol ||B_t||.  bnorm2 of the group's k columns becomes
// min_t allowance_t^2 / (k tol^2) over frames with B_t != 0, since the test
// on column j is ||rho_j||^2 <= tol^2 bnorm2[j] (unchanged if there is none).
__global__ void __launch_bounds__(kBlock)
k_group_ref(const uint8_t* __restrict__ records, SeqLayout sl, int nc, int nz, int ncols,
            int nchunks, int kk2, const int32_t* __restrict__ anchors,
            const double* __restrict__ ut, const double* __restrict__ b,
            const double* __restrict__ Ah,
            const double* __restrict__ part, double g_resid, double tol,
            double* __restrict__ bnorm2) {
  __shared__ double gram[1024];
  __shared__ double sbA[64 * 33];   // anchor rows of b: [anchor of the chunk][r]
  __shared__ double sAh[64 * 65];   // A^ of the chunk: [anchor][t]; then s_t[r] at [t][r] (33)
  const int g = blockIdx.x, w = g / 3, c = g % 3;
  const uint8_t* rec;
  int T, k, t0;
  RecordLayout lay;
  window_of(sl, records, w, rec, T, k, t0, lay);
  const int col0 = zoff(sl, w) + c * k;
  const int tid = threadIdx.x;
  // Gram matrix: the partials in order, four independent sums
  for (int e = tid; e < k * k; e += kBlock) {
    const double* pe = part + (size_t)g * nchunks * kk2 + e;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int q = 0;
    for (; q + 3 < nchunks; q += 4) {
      a0 += pe[(size_t)q * kk2];
      a1 += pe[(size_t)(q + 1) * kk2];
      a2 += pe[(size_t)(q + 2) * kk2];
      a3 += pe[(size_t)(q + 3) * kk2];
    }
    for (; q < nchunks; ++q) a0 += pe[(size_t)q * kk2];
    gram[e] = (a0 + a1) + (a2 + a3);
  }
  // s_t[r] = sum_a b[anchor_a][col0 + r] A^[a][t] (thread owns entries tid + 256 u of
  // the T x k block, T k <= 2048), ||A^_t||^2 and ||A^_t||_1 (threads t < T)
  double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  double an2 = 0.0, an1 = 0.0;
  for (int a0 = 0; a0 < nc; a0 += 64) {
    const int na = min(64, nc - a0);
    __syncthreads();
    for (int e = tid; e < na * k; e += kBlock) {
      const int a = e / k, r = e % k;
      sbA[a * 33 + r] = b[(size_t)anchors[a0 + a] * nz + col0 + r];
    }
    for (int e = tid; e < na * T; e += kBlock) {
      const int a = e / T, t = e % T;
      sAh[a * 65 + t] = Ah[(size_t)(a0 + a) * ncols + 3 * (t0 + t) + c];
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = tid + u * kBlock;
      if (e < T * k) {
        const int t = e / k, r = e % k;
        double s = acc[u];
        for (int a = 0; a < na; ++a) s = fma(sbA[a * 33 + r], sAh[a * 65 + t], s);
        acc[u] = s;
      }
    }
    if (tid < T)
      for (int a = 0; a < na; ++a) {
        const double v = sAh[a * 65 + tid];
        an2 = fma(v, v, an2);
        an1 += fabs(v);
      }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int e = tid + u * kBlock;
    if (e < T * k) sAh[(e / k) * 33 + e % k] = acc[u];
  }
  __syncthreads();
  if (tid >= 64) return;  // T <= 64: the frames are in the first wavefront
  const int t = tid;
  double allow2 = -1.0;  // < 0: frame without content
  if (t < T) {
    const double* ud = dict_of(sl, ut, w);
    double u[32];
#pragma unroll
    for (int r = 0; r < 32; ++r) u[r] = r >= k ? 0.0 : ud[(c * T + t) * k + r];
    double q = an2;
#pragma unroll
    for (int r = 0; r < 32; ++r) {
      if (r >= k) continue;
      double gu = 0.0;
#pragma unroll
      for (int s = 0; s < 32; ++s)
        if (s < k) gu = fma(gram[r * k + s], u[s], gu);
      q += u[r] * gu + 2.0 * u[r] * sAh[t * 33 + r];
    }
    const double bn = sqrt(fmax(q, 0.0));
    if (bn > 0.0) {
      const double allow = tol * bn - g_resid * an1;
      allow2 = allow > 0.0 ? allow * allow : 0.0;
    }
  }
  // smallest allowance over the frames with content
  const double m = wave_min(allow2 >= 0.0 ? allow2 : 1e308);
  if (m < 1e308 && t < k) bnorm2[col0 + t] = fmax(m, 1e-300) / ((double)k * tol * tol);
}

constexpr int CP_V = 64;  // vertices per compose block and vertex tile (16 per wavefront)

// frames of window w for 64 vertices, coordinate by coordinate:
//   X_c^T (T x 16 vertices) = A^_c^T G^T + U~_c Z_c^T,
// i.e. X[i][t][c] = sum_a A^[a][3(t0 + t) + c] G[i][a] + sum_r U~_c[t][r] Z[i][zoff + c k + r],
// on the FP64 matrix cores.  Each wavefront owns 16 vertices and reads its
// operand fragments straight from memory (G, Z rows of its vertices; A^ and
// the dictionary, shared by every wavefront, from the caches): no LDS, no
// barriers.  v_mfma_f64_16x16x4f64: lane l supplies A[l%16][l/16] (frame,
// K index) and B[l/16][l%16] (K index, vertex); component r of lane l is
// D[4r + l/16][l%16], so a store covers 16 consecutive vertices.
// TTM: 16-frame tiles held (2 for T <= 32, 4 for T <= 64).
// The compose products in the output's type: float64 frames on the FP64
// matrix cores; float32 frames on the FP32 ones (v_mfma_f32_16x16x4f32, the
// same operand layout, twice the rate; the products' rounding, ~1e-7
// relative, is that of the float32 output itself).
typedef float cf4 __attribute__((ext_vector_type(4)));
template <typename Real>
struct ComposeMfma;
// Component r of lane l holds result row row(r, l / 16), column l % 16: the
// FP64 instruction interleaves the rows (4 r + l / 16), the FP32 one gives
// each group of 16 lanes four consecutive rows (4 (l / 16) + r).
template <>
struct ComposeMfma<double> {
  using Acc = d4;
  __device__ static Acc step(double a, double b, Acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int r, int q) { return 4 * r + q; }
};
template <>
struct ComposeMfma<float> {
  using Acc = cf4;
  __device__ static Acc step(double a, double b, Acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32((float)a, (float)b, c, 0, 0, 0);
  }
  __device__ static int row(int r, int q) { return 4 * q + r; }
};

template <typename Real, int TTM, int NV>
__global__ void __launch_bounds__(kBlock)
k_compose(const uint8_t* __restrict__ records, SeqLayout sl, int n, int nc, int nz, int ncols,
          const int32_t* __restrict__ pos, const double* __restrict__ G,
          const double* __restrict__ Z, const double* __restrict__ Ah,
          const double* __restrict__ ut, Real* __restrict__ out) {
  const int w = blockIdx.y;
  const uint8_t* rec;
  int T, k, t0;
  RecordLayout lay;
  window_of(sl, records, w, rec, T, k, t0, lay);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  // this lane's vertices (B columns), one per 16-vertex tile of the wavefront
  int iv_[NV], ip_[NV];  // vertex, and its row in G and Z
  bool ok_[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    iv_[v] = (blockIdx.x * 4 + wv) * 16 * NV + 16 * v + lane % 16;
    ok_[v] = iv_[v] < n;
    ip_[v] = ok_[v] ? pos[iv_[v]] : 0;
  }
  const int kq = lane / 16;  // K index within a step of four
  const int tl = lane % 16;  // frame within a 16-frame tile (A row)
  const int tt_n = (T + 15) / 16;
  const int z0 = zoff(sl, w);
  const double* ud = dict_of(sl, ut, w);
  using Acc = typename ComposeMfma<Real>::Acc;
  Acc acc[3][TTM][NV];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int tt = 0; tt < TTM; ++tt)
#pragma unroll
      for (int v = 0; v < NV; ++v) acc[c][tt][v] = Acc{0, 0, 0, 0};
  // Operands are read without branches: indices past an edge are clamped to
  // an element that exists and the value is replaced by zero afterwards
  // (frames past T too, whose sums are never stored).  The operands of CS K
  // steps are loaded, then pinned (pin: the compiler would otherwise move
  // each load behind its bounds test and wait on them one by one), then
  // multiplied, so their loads are in flight together.  Every accumulator
  // still takes its K steps in order.
  constexpr int CS = 2;
  // anchor part: K = anchors, four per step
  for (int a00 = 0; a00 < nc; a00 += 4 * CS) {
    double vb[CS][NV], va[CS][3][TTM];
#pragma unroll
    for (int g = 0; g < CS; ++g) {
      const int ac = min(a00 + 4 * g + kq, nc - 1);
#pragma unroll
      for (int v = 0; v < NV; ++v) vb[g][v] = G[(size_t)ip_[v] * nc + ac];
      const double* ar = Ah + (size_t)ac * ncols + 3 * t0;
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int tt = 0; tt < TTM; ++tt) va[g][c][tt] = ar[3 * min(16 * tt + tl, T - 1) + c];
    }
#pragma unroll
    for (int g = 0; g < CS; ++g) {
      const bool av = a00 + 4 * g + kq < nc;
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        pin(vb[g][v]);
        vb[g][v] = (ok_[v] && av) ? vb[g][v] : 0.0;
      }
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int tt = 0; tt < TTM; ++tt) {
          pin(va[g][c][tt]);
          va[g][c][tt] = (av && 16 * tt + tl < T) ? va[g][c][tt] : 0.0;
        }
    }
#pragma unroll
    for (int g = 0; g < CS; ++g)
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int tt = 0; tt < TTM; ++tt)
#pragma unroll
          for (int v = 0; v < NV; ++v)
            acc[c][tt][v] = ComposeMfma<Real>::step(va[g][c][tt], vb[g][v], acc[c][tt][v]);
  }
  // subspace part: K = the k coefficients of each coordinate
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    for (int r00 = 0; r00 < k; r00 += 4 * CS) {
      double vb[CS][NV], va[CS][TTM];
#pragma unroll
      for (int g = 0; g < CS; ++g) {
        const int rc = min(r00 + 4 * g + kq, k - 1);
#pragma unroll
        for (int v = 0; v < NV; ++v) vb[g][v] = Z[(size_t)ip_[v] * nz + z0 + c * k + rc];
#pragma unroll
        for (int tt = 0; tt < TTM; ++tt)
          va[g][tt] = ud[(c * T + min(16 * tt + tl, T - 1)) * k + rc];
      }
#pragma unroll
      for (int g = 0; g < CS; ++g) {
        const bool rv = r00 + 4 * g + kq < k;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          pin(vb[g][v]);
          vb[g][v] = (ok_[v] && rv) ? vb[g][v] : 0.0;
        }
#pragma unroll
        for (int tt = 0; tt < TTM; ++tt) {
          pin(va[g][tt]);
          va[g][tt] = (rv && 16 * tt + tl < T) ? va[g][tt] : 0.0;
        }
      }
#pragma unroll
      for (int g = 0; g < CS; ++g)
#pragma unroll
        for (int tt = 0; tt < TTM; ++tt)
#pragma unroll
          for (int v = 0; v < NV; ++v)
            acc[c][tt][v] = ComposeMfma<Real>::step(va[g][tt], vb[g][v], acc[c][tt][v]);
    }
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    if (!ok_[v]) continue;
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int tt = 0; tt < TTM; ++tt)
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
          const int t = 16 * tt + ComposeMfma<Real>::row(rr, kq);
          if (tt < tt_n && t < T)
            out[((size_t)(t0 + t) * n + iv_[v]) * 3 + c] = (Real)acc[c][tt][v][rr];
        }
  }
}

}  // namespace

// grid of k_rhs: row blocks padded to the XCD count, 256-column tiles
static dim3 rhs_grid(int n, int ncols) {
  return dim3(pad_xcd((n + CG_RB - 1) / CG_RB), (ncols + SP_CW - 1) / SP_CW);
}

size_t cg_part_rows(int32_t n) { return (size_t)(n + CG_RB - 1) / CG_RB; }

void launch_dict_decode(hipStream_t s, const uint8_t* records, const SeqLayout& sl, double* ut) {
  // full windows (in order in one block when a column may refer to its
  // predecessor), then the short last window (values only)
  const RecordLayout& f = sl.full;
  const bool chained = f.dict_mode == DMC_DICT_ADAPTIVE;
  auto launch = [&](const uint8_t* rec, size_t rec_bytes, const RecordLayout& l, int nw,
                    double* out) {
    if (nw < 1) return;
    const int per = chained ? nw : 1;
    const dim3 grid(chained ? 1 : nw);
    if (l.precision == DMC_FP64)
      hipLaunchKernelGGL(k_dict_decode<double>, grid, dim3(kBlock), 0, s, rec, rec_bytes, l, nw,
                         per, out);
    else
      hipLaunchKernelGGL(k_dict_decode<float>, grid, dim3(kBlock), 0, s, rec, rec_bytes, l, nw,
                         per, out);
  };
  launch(records, sl.rec_bytes_full, f, sl.nw_full, ut);
  if (sl.T_tail)
    launch(records + (size_t)sl.nw_full * sl.rec_bytes_full, sl.tail.bytes, sl.tail, 1,
           ut + (size_t)sl.nw_full * 3 * sl.T * f.k);
}

size_t dict_decode_doubles(const SeqLayout& sl) {
  return (size_t)(sl.nw_full + (sl.T_tail > 0 ? 1 : 0)) * 3 * sl.T * sl.full.k;
}

// z = M^-1 r by the Cholesky factor and the r.z partials; with p_out the
// solve writes straight into p_out (the first search direction p = z; z
// itself is rewritten by every later application before it is read)
void launch_precond_apply(hipStream_t s, const MeshDev& m, int32_t ncols, const CgBuffers& cb,
                          double* p_out) {
  const int nrb = (int)cg_part_rows(m.n);
  dim3 grid(nrb, (ncols + SP_COLS - 1) / SP_COLS);
  double* z = p_out ? p_out : cb.z;
  launch_chol_solve(s, m.chol, ncols, cb.r, z, cb.W, cb.Y, cb.U, cb.S, cb.split_target);
  hipLaunchKernelGGL(k_cg_dot, grid, dim3(kBlock), 0, s, m.n, ncols, cb.r, z, (double*)nullptr,
                     cb.part);
}

void launch_cg_init(hipStream_t s, const MeshDev& m, int32_t ncols, const double* b,
                    const CgBuffers& cb, int32_t precond, bool zero_x, bool bb_done) {
  const int nrb = (int)cg_part_rows(m.n);
  dim3 grid(nrb, (ncols + kBlock - 1) / kBlock);
  // with the Cholesky preconditioner, b built in place in r and x left to
  // the first update, the init kernel's only remaining output is the b.b
  // partials, which the right-hand-side kernel has already written
  const bool skip = bb_done && precond == DMC_PRECOND_CHOLESKY && !zero_x && b == cb.r;
  if (!skip)
    hipLaunchKernelGGL(k_cg_init, grid, dim3(kBlock), 0, s, b, m.m_dinv, precond, zero_x ? 1 : 0,
                       m.n, ncols, cb.x, cb.r, cb.p, cb.part);
  if (precond == DMC_PRECOND_CHOLESKY) launch_precond_apply(s, m, ncols, cb, cb.p);
  hipLaunchKernelGGL(k_cg_init_reduce, dim3((ncols + RED_COLS - 1) / RED_COLS, 2), dim3(kBlock), 0, s,
                     cb.part, nrb, ncols, cb.bnorm2, cb.rz, cb.done, cb.resid);
}

void launch_cg_norms(hipStream_t s, const MeshDev& m, int32_t ncols, const CgBuffers& cb) {
  const int nrb = (int)cg_part_rows(m.n);
  hipLaunchKernelGGL(k_cg_init_reduce, dim3((ncols + RED_COLS - 1) / RED_COLS, 1), dim3(kBlock), 0,
                     s, cb.part, nrb, ncols, cb.bnorm2, cb.rz, cb.done, cb.resid);
}

// k_cg_residual with two columns per lane when the column count is even
// (the vectors' rows then start at 16-byte boundaries), else one
static void launch_residual(hipStream_t s, const MeshDev& m, int32_t ncols, const double* x,
                            double* b, int write_r, double* part) {
  const int nrbp = pad_xcd((int)cg_part_rows(m.n));
  if (ncols % 2 == 0)
    hipLaunchKernelGGL(k_cg_residual<2>, dim3(nrbp, (ncols + 127) / 128), dim3(kBlock), 0, s,
                       m.m_rowptr, m.m_col, m.m_val, m.n, ncols, x, b, write_r, part);
  else
    hipLaunchKernelGGL(k_cg_residual<1>, dim3(nrbp, (ncols + 63) / 64), dim3(kBlock), 0, s,
                       m.m_rowptr, m.m_col, m.m_val, m.n, ncols, x, b, write_r, part);
}

void launch_cg_warm_start(hipStream_t s, const MeshDev& m, int32_t ncols, const CgBuffers& cb,
                          double tol) {
  const int nrb = (int)cg_part_rows(m.n);
  dim3 cgrid((ncols + RED_COLS - 1) / RED_COLS);
  launch_chol_solve(s, m.chol, ncols, cb.r, cb.x, cb.W, cb.Y, cb.U, cb.S, cb.split_target);
  prof::begin(s, DMC_KERNEL_CG_SPMM);
  launch_residual(s, m, ncols, cb.x, cb.r, 0, cb.part);
  prof::end(s, DMC_KERNEL_CG_SPMM);
  hipLaunchKernelGGL(k_cg_resid, cgrid, dim3(kBlock), 0, s, cb.part, nrb, ncols, cb.bnorm2,
                     cb.done, cb.resid, tol);
}

void launch_cg_restart(hipStream_t s, const MeshDev& m, int32_t ncols, const CgBuffers& cb) {
  const int nrb = (int)cg_part_rows(m.n);
  prof::begin(s, DMC_KERNEL_CG_SPMM);
  launch_residual(s, m, ncols, cb.x, cb.r, 1, cb.part);
  prof::end(s, DMC_KERNEL_CG_SPMM);
  launch_precond_apply(s, m, ncols, cb, cb.p);
  hipLaunchKernelGGL(k_cg_rz_reduce, dim3((ncols + RED_COLS - 1) / RED_COLS), dim3(kBlock), 0, s,
                     cb.part, nrb, ncols, cb.rz);
}

void launch_cg_step_a(hipStream_t s, const MeshDev& m, int32_t ncols, const CgBuffers& cb,
                      int32_t precond, double tol, bool first) {
  const int nrb = (int)cg_part_rows(m.n);
  dim3 sgrid(nrb, (ncols + SP_COLS - 1) / SP_COLS);
  const dim3 xgrid(pad_xcd(nrb), sgrid.y);  // k_cg_spmm
  dim3 cgrid((ncols + RED_COLS - 1) / RED_COLS);
  prof::begin(s, DMC_KERNEL_CG_SPMM);
  hipLaunchKernelGGL(k_cg_spmm, xgrid, dim3(kBlock), 0, s, m.m_rowptr, m.m_col, m.m_val, m.n,
                     ncols, cb.p, cb.q, cb.part);
  prof::end(s, DMC_KERNEL_CG_SPMM);
  hipLaunchKernelGGL(k_cg_alpha, cgrid, dim3(kBlock), 0, s, cb.part, nrb, ncols, cb.rz, cb.done,
                     cb.alpha);
  prof::begin(s, DMC_KERNEL_CG_UPDATE);
  hipLaunchKernelGGL(k_cg_update, sgrid, dim3(kBlock), 0, s, m.n, ncols, cb.alpha, m.m_dinv,
                     precond, first ? 1 : 0, cb.x, cb.r, cb.p, cb.q, cb.part);
  prof::end(s, DMC_KERNEL_CG_UPDATE);
  hipLaunchKernelGGL(k_cg_resid, cgrid, dim3(kBlock), 0, s, cb.part, nrb, ncols, cb.bnorm2,
                     cb.done, cb.resid, tol);
}

namespace {
// out[0] = largest relative residual over the columns, out[1] = 1 if every
// column has converged (else 0)
__global__ void __launch_bounds__(kBlock)
k_cg_summary(const double* __restrict__ resid, const int32_t* __restrict__ done, int ncols,
             double* __restrict__ out) {
  __shared__ double smax[kBlock];
  __shared__ int sdone[kBlock];
  double m = 0.0;
  int d = 1;
  for (int j = threadIdx.x; j < ncols; j += kBlock) {
    m = fmax(m, resid[j]);
    d = d && (done[j] != 0);
  }
  smax[threadIdx.x] = m;
  sdone[threadIdx.x] = d;
  __syncthreads();
  for (int st = kBlock / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) {
      smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + st]);
      sdone[threadIdx.x] = sdone[threadIdx.x] && sdone[threadIdx.x + st];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = smax[0];
    out[1] = sdone[0] ? 1.0 : 0.0;
  }
}
}  // namespace

void launch_cg_summary(hipStream_t s, const CgBuffers& cb, int32_t ncols, double* out) {
  hipLaunchKernelGGL(k_cg_summary, dim3(1), dim3(kBlock), 0, s, cb.resid, cb.done, ncols, out);
}

void launch_cg_step_b(hipStream_t s, const MeshDev& m, int32_t ncols, const CgBuffers& cb,
                      int32_t precond) {
  const int nrb = (int)cg_part_rows(m.n);
  dim3 grid(nrb, (ncols + kBlock - 1) / kBlock);
  dim3 cgrid((ncols + RED_COLS - 1) / RED_COLS);
  if (precond == DMC_PRECOND_CHOLESKY) launch_precond_apply(s, m, ncols, cb, nullptr);
  hipLaunchKernelGGL(k_cg_beta, cgrid, dim3(kBlock), 0, s, cb.part, nrb, ncols, cb.rz, cb.done,
                     cb.beta);
  hipLaunchKernelGGL(k_cg_pupdate, grid, dim3(kBlock), 0, s, m.n, ncols, cb.beta, m.m_dinv,
                     precond, cb.r, cb.z, cb.p);
}

void launch_to_frames(hipStream_t s, const MeshDev& m, const double* X, int32_t F,
                      int32_t precision, void* frames_out) {
  const int n = m.n;
  dim3 grid((n + TF_V - 1) / TF_V, (F + TF_T - 1) / TF_T);
  prof::begin(s, DMC_KERNEL_TO_FRAMES);
  if (precision == DMC_FP64)
    hipLaunchKernelGGL(k_to_frames<double>, grid, dim3(kBlock), 0, s, X, m.dpos, n, F,
                       (double*)frames_out);
  else
    hipLaunchKernelGGL(k_to_frames<float>, grid, dim3(kBlock), 0, s, X, m.dpos, n, F,
                       (float*)frames_out);
  prof::end(s, DMC_KERNEL_TO_FRAMES);
}


int32_t reduced_cols(const SeqLayout& sl) {
  return 3 * (sl.full.k * sl.nw_full + (sl.T_tail > 0 ? sl.tail.k : 0));
}

void launch_coef_rows(hipStream_t s, const MeshDev& m, const uint8_t* records,
                      const SeqLayout& sl, double* Yd) {
  const int nw = sl.nw_full + (sl.T_tail > 0 ? 1 : 0);
  dim3 grid((m.n + CR_V - 1) / CR_V, nw);
  const int nz = reduced_cols(sl);
  prof::begin(s, DMC_KERNEL_BACK_PROJECT);
  if (sl.full.precision == DMC_FP64)
    hipLaunchKernelGGL(k_coef_rows<double>, grid, dim3(kBlock), 0, s, records, sl, m.n, nz,
                       m.dpos, Yd);
  else
    hipLaunchKernelGGL(k_coef_rows<float>, grid, dim3(kBlock), 0, s, records, sl, m.n, nz,
                       m.dpos, Yd);
  prof::end(s, DMC_KERNEL_BACK_PROJECT);
}

void launch_rhs_reduced(hipStream_t s, const MeshDev& m, int32_t nz, const double* Yd, double* b,
                        double* bb) {
  const dim3 grid = rhs_grid(m.n, nz);
  prof::begin(s, DMC_KERNEL_RHS);
  hipLaunchKernelGGL(k_rhs, grid, dim3(kBlock), 0, s, m.d_rowptr, m.d_col, m.d_w64,
                     m.laplacian == DMC_LAP_UNIFORM ? 1 : 0, m.d_slot, m.n, nz, (int)grid.x, Yd,
                     (const double*)nullptr, b, bb);
  prof::end(s, DMC_KERNEL_RHS);
}

void launch_rhs_from_coefs(hipStream_t s, const MeshDev& m, const SeqLayout& sl,
                           const double* Yd, const double* ut, const double* Ah, double* b,
                           double* bb) {
  const int nw = sl.nw_full + (sl.T_tail > 0 ? 1 : 0);
  const int F = sl.nw_full * sl.T + sl.T_tail;
  const dim3 grid(pad_xcd((m.n + CG_RB - 1) / CG_RB), nw);
  auto kern = sl.full.k > 16 ? k_rhs_expand<32> : k_rhs_expand<16>;
  prof::begin(s, DMC_KERNEL_RHS);
  hipLaunchKernelGGL(kern, grid, dim3(kBlock), 0, s, m.d_rowptr, m.d_col, m.d_w64,
                     m.laplacian == DMC_LAP_UNIFORM ? 1 : 0, m.d_slot, m.n, 3 * F,
                     reduced_cols(sl), (int)grid.x, sl, Yd, ut, Ah, b, bb);
  prof::end(s, DMC_KERNEL_RHS);
}

void launch_anchor_values(hipStream_t s, const MeshDev& m, const uint8_t* records,
                          const SeqLayout& sl, double* Ah) {
  const int F = sl.nw_full * sl.T + sl.T_tail;
  const int ncols = 3 * F;
  const size_t tot = (size_t)m.nc * ncols;
  if (tot == 0) return;
  if (sl.full.precision == DMC_FP64)
    hipLaunchKernelGGL(k_anchor_values<double>, dim3((tot + kBlock - 1) / kBlock), dim3(kBlock),
                       0, s, records, sl, m.nc, ncols, Ah);
  else
    hipLaunchKernelGGL(k_anchor_values<float>, dim3((tot + kBlock - 1) / kBlock), dim3(kBlock), 0,
                       s, records, sl, m.nc, ncols, Ah);
}

size_t group_gram_doubles(int32_t n, const SeqLayout& sl) {
  const int nw = sl.nw_full + (sl.T_tail > 0 ? 1 : 0);
  const int nchunks = (n + GR_ROWS - 1) / GR_ROWS;
  return (size_t)3 * nw * nchunks * sl.full.k * sl.full.k;
}

void launch_group_ref(hipStream_t s, const MeshDev& m, const uint8_t* records, const SeqLayout& sl,
                      const double* ut, const double* b, const double* Ah, double tol,
                      double* gram_part, double* bnorm2) {
  if (!(tol > 0.0)) return;
  const int nw = sl.nw_full + (sl.T_tail > 0 ? 1 : 0);
  const int nchunks = (m.n + GR_ROWS - 1) / GR_ROWS;
  const int nz = reduced_cols(sl);
  const int F = sl.nw_full * sl.T + sl.T_tail;
  const int kk2 = sl.full.k * sl.full.k;
  hipLaunchKernelGGL(k_group_gram, dim3(3 * nw, nchunks), dim3(kBlock), 0, s, sl, m.n, nz, kk2, b,
                     gram_part);
  hipLaunchKernelGGL(k_group_ref, dim3(3 * nw), dim3(kBlock), 0, s, records, sl, m.nc, nz, 3 * F,
                     nchunks, kk2, m.d_anchors, ut, b, Ah, (const double*)gram_part, m.G_resid, tol,
                     bnorm2);
}

void launch_anchor_unit_rhs(hipStream_t s, const MeshDev& m, double* b) {
  const size_t tot = (size_t)m.n * m.nc;
  hipLaunchKernelGGL(k_anchor_unit_rhs, dim3((tot + kBlock - 1) / kBlock), dim3(kBlock), 0, s,
                     m.d_slot, m.n, m.nc, b);
}

void launch_compose(hipStream_t s, const MeshDev& m, const uint8_t* records, const SeqLayout& sl,
                    const double* ut, const double* Z, const double* Ah, int32_t precision,
                    void* frames_out) {
  const int nw = sl.nw_full + (sl.T_tail > 0 ? 1 : 0);
  const int F = sl.nw_full * sl.T + sl.T_tail;
  const int nz = reduced_cols(sl);
  prof::begin(s, DMC_KERNEL_TO_FRAMES);
  // T <= 32: two 16-vertex tiles per wavefront, so each anchor-value and
  // dictionary operand serves two products (the same accumulator count as
  // T <= 64 with one tile)
  const bool t32 = sl.T <= 32;  // the tail window is never longer
  const int nv = t32 ? 2 : 1;
  dim3 grid((m.n + CP_V * nv - 1) / (CP_V * nv), nw);
  if (precision == DMC_FP64) {
    auto kern = t32 ? k_compose<double, 2, 2> : k_compose<double, 4, 1>;
    hipLaunchKernelGGL(kern, grid, dim3(kBlock), 0, s, records, sl, m.n, m.nc, nz, 3 * F, m.dpos,
                       m.G, Z, Ah, ut, (double*)frames_out);
  } else {
    auto kern = t32 ? k_compose<float, 2, 2> : k_compose<float, 4, 1>;
    hipLaunchKernelGGL(kern, grid, dim3(kBlock), 0, s, records, sl, m.n, m.nc, nz, 3 * F, m.dpos,
                       m.G, Z, Ah, ut, (float*)frames_out);
  }
  prof::end(s, DMC_KERNEL_TO_FRAMES);
}

}  // namespace dmc
