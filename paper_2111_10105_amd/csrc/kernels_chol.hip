// Supernodal triangular solves with the Cholesky factor of the normal matrix
// (the decoder's preconditioner): z = (L L^T)^{-1} r for every column at once.
// r and z hold their rows in elimination order (the decoder keeps all its
// n-row blocks in that order), so the solves read and write them in place.
//
// Each supernode s (columns a..a+w-1, rows R_s of size m) carries the solve
// operator B_s = [inv(L_ss); L_os inv(L_ss)] (m x w), precomputed on the host.
// Level scheduling over the supernodal tree (supernodes of one level are
// independent):
//   forward, level 0 upwards
//     gather : W_s = r[rows of s] - sum of the update rows aimed at s
//     gemm   : [Y_s; U_s] = B_s W_s   (Y_s = solution rows, U_s = update rows
//              for the ancestors, one slot per row of s below its diagonal block)
//   backward, top level downwards
//     gemm   : z_s = B_s^T [Y_s; -z_(R_s below the diagonal block)]
// Work items are (supernode, 64-row tile) x 64-column tiles (the gather splits
// each tile into four blocks of 16 rows; the backward GEMM splits its K range
// over several blocks on levels with few tiles, and a second kernel adds the
// partial sums in a fixed order).  The two GEMMs
// stage shallow K slices (16 deep forward, 4 backward) of B_s and of the
// right-hand rows in LDS and run on
// the FP64 matrix cores; the gather is one load per update row.
#include "dmc_internal.h"

namespace dmc {
namespace {

constexpr int CTG = 64;  // columns per gather / reduce block (one per lane)

// Block order of every solve kernel: column tiles fastest, block b = ct +
// cbp (u + nu v), with cbp (the column-tile count padded to a multiple of
// the 8 XCDs) so that the dispatcher, which deals consecutive blocks to the
// XCDs in turn, runs every block of column tile ct on XCD ct mod 8.  A
// tile's right-hand and solution rows then stay in that XCD's L2 from row
// tile to row tile and level to level, and the blocks of one operator tile
// run together, one read of it per XCD.  Blocks of padding tiles (ct >= the
// tile count) return at once.

struct ColBlock {
  int ct, u, v;
};
__device__ inline ColBlock col_block(int cbp, int nu) {
  const int b = blockIdx.x, q = b / cbp;
  return {b % cbp, q % nu, q / nu};
}
constexpr int RTK = 64;  // rows per task of the task lists
constexpr int GQ = 16;   // gather: blocks per task (4 rows each, one per wave)
constexpr int RPW = RTK / GQ / (kBlock / 64);  // gather rows per wave

__global__ void __launch_bounds__(kBlock)
k_fwd_gather(CholDev f, int t0, int ncols, int cbp, const double* __restrict__ rhs,
             const double* __restrict__ U, double* __restrict__ W) {
  const ColBlock cbk = col_block(cbp, GQ);  // u = quarter, v = task
  const int task = t0 + cbk.v;
  const int s = f.task_w_sn[task], r0 = f.task_w_r0[task];
  const int c = cbk.ct * CTG + threadIdx.x % CTG;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
  if (c >= ncols) return;
  const int a = f.sn_start[s], w = f.sn_start[s + 1] - a;
  for (int k = 0; k < RPW; ++k) {
    const int t = r0 + cbk.u * (RTK / GQ) + wv * RPW + k;
    if (t >= w) break;
    const int j = a + t;
    double acc = rhs[(size_t)j * ncols + c];
    const int e1 = f.contrib_ptr[j + 1];
    int e = f.contrib_ptr[j];
    // eight independent partial sums keep several loads in flight
    double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (; e + 8 <= e1; e += 8)
#pragma unroll
      for (int q = 0; q < 8; ++q) a[q] -= U[(size_t)f.contrib_slot[e + q] * ncols + c];
    for (; e < e1; ++e) acc -= U[(size_t)f.contrib_slot[e] * ncols + c];
    W[(size_t)j * ncols + c] = acc + (((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7])));
  }
}

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int RIDX = 2048;   // ancestor row indices cached per block
// LDS stages of the solve GEMMs: one stage (the next chunk waits in registers
// while the current one is multiplied, then replaces it after a barrier)
// halves the LDS of a block, so twice the blocks share a CU and cover each
// other's load latency.
constexpr int kStages = 1;
// K chunk depth of the forward and backward GEMMs (the backward one at least
// kBlock / RT, one element per thread)
constexpr int kKcFwd = 16;
constexpr int kKcBwd = 4;
constexpr int bwd_kc(int rt) { return rt * kKcBwd >= kBlock ? kKcBwd : kBlock / rt; }

// One RT x RT output tile per block on the FP64 matrix cores (RT = 64 or 32):
// wave v owns the quadrant (v / 2, v % 2) as NQ x NQ tiles of
// v_mfma_f64_16x16x4f64 (NQ = RT / 32; lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; component r of lane l is D[4r + l/16][l%16]).  The 32 x 32
// tiles serve forward levels with few tasks: four times the blocks, a quarter
// of the matrix-core work on each block's critical path.  K chunks are KC_
// deep: shallow chunks keep a block's LDS small (more blocks per CU to cover
// each other's loads) and pad the short K ranges of the leaves less.
template <int RT, int KC_>
struct MfmaTile {
  static constexpr int NQ = RT / 32, LDB = RT + 1;
  static constexpr int KC = KC_, LDA = KC + 1;
  static_assert(KC % 4 == 0 && RT * KC % kBlock == 0, "a chunk is whole MFMA steps, whole per thread");
  d4 acc[NQ][NQ];
  __device__ void zero() {
#pragma unroll
    for (int a = 0; a < NQ; ++a)
#pragma unroll
      for (int b = 0; b < NQ; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
  }
  __device__ void step(const double* As, const double* Bs, int wr, int wc, int lane) {
#pragma unroll
    for (int kk = 0; kk < KC; kk += 4) {
      double af[NQ], bf[NQ];
#pragma unroll
      for (int a = 0; a < NQ; ++a)
        af[a] = As[(wr * 16 * NQ + a * 16 + lane % 16) * LDA + kk + lane / 16];
#pragma unroll
      for (int b = 0; b < NQ; ++b)
        bf[b] = Bs[(kk + lane / 16) * LDB + wc * 16 * NQ + b * 16 + lane % 16];
#pragma unroll
      for (int a = 0; a < NQ; ++a)
#pragma unroll
        for (int b = 0; b < NQ; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a], bf[b], acc[a][b], 0, 0, 0);
    }
  }
};

// The task of a block: the 64-row task lists are shared by both tile sizes;
// with RT = 32 block x takes half x % 2 of task x / 2 (rows r0 + 32 (x % 2)).
template <int RT>
__device__ inline int tile_task(int t0, int tidx, int& half) {
  if (RT == 64) {
    half = 0;
    return t0 + tidx;
  }
  half = tidx & 1;
  return t0 + (tidx >> 1);
}

// forward: [Y_s; U_s] rows r0..r0+RT-1 = B_s W_s (K = columns of B_s; rows of the
// diagonal block only need the lower triangle of inv(L_ss)).  The global
// loads of chunk j+1 are in flight (in registers) while chunk j is multiplied
// out of the LDS stage (kStages).
template <int RT>
__global__ void __launch_bounds__(kBlock)
k_fwd_gemm(CholDev f, int t0, int ncols, int cbp, int ntile, const double* __restrict__ W,
           double* __restrict__ Y, double* __restrict__ U) {
  using Tile = MfmaTile<RT, kKcFwd>;
  constexpr int CT = RT, LDB = Tile::LDB;
  constexpr int KC = Tile::KC, LDA = Tile::LDA;
  constexpr int PER_T = RT * KC / kBlock;  // elements of a chunk staged per thread
  __shared__ double As[kStages][RT * LDA];
  __shared__ double Bs[kStages][KC * LDB];
  const ColBlock cbk = col_block(cbp, ntile);  // u = row tile
  if (cbk.ct * CT >= ncols) return;           // padding tile: whole block
  int half;
  const int task = tile_task<RT>(t0, cbk.u, half);
  const int s = f.task_m_sn[task], r0 = f.task_m_r0[task] + RT * half;
  const int a = f.sn_start[s], w = f.sn_start[s + 1] - a;
  const int m = f.sn_rowptr[s + 1] - f.sn_rowptr[s];
  if (r0 >= m) return;  // whole block
  const int c0 = cbk.ct * CT;
  const double* Br = f.brow + f.sn_valptr[s];
  const int tid = threadIdx.x, lane = tid % 64, wv = tid / 64;
  const int wr = wv / 2, wc = wv % 2;
  const int qend = r0 + RT <= w ? r0 + RT : w;
  double ra[PER_T], rb[PER_T];
  auto load = [&](int q0) {
#pragma unroll
    for (int u = 0; u < PER_T; ++u) {
      const int e = tid + u * kBlock;
      const int ii = e / KC, qq = e % KC;
      const int i = r0 + ii, q = q0 + qq;
      ra[u] = (i < m && q < qend) ? Br[(size_t)i * w + q] : 0.0;
      const int q2 = e / CT, cc = e % CT;
      const int qb = q0 + q2, c = c0 + cc;
      rb[u] = (qb < qend && c < ncols) ? W[(size_t)(a + qb) * ncols + c] : 0.0;
    }
  };
  auto store = [&](int st) {
#pragma unroll
    for (int u = 0; u < PER_T; ++u) {
      const int e = tid + u * kBlock;
      As[st][(e / KC) * LDA + e % KC] = ra[u];
      Bs[st][(e / CT) * LDB + e % CT] = rb[u];
    }
  };
  Tile t;
  t.zero();
  int st = 0;
  if (qend > 0) {
    load(0);
    store(0);
  }
  __syncthreads();
  for (int q0 = 0; q0 < qend; q0 += KC) {
    const bool more = q0 + KC < qend;
    if (more) load(q0 + KC);
    t.step(As[st], Bs[st], wr, wc, lane);
    if (more) {
      if (kStages == 1) __syncthreads();  // every wave has read the stage
      store(kStages == 1 ? 0 : st ^ 1);
    }
    __syncthreads();
    if (kStages == 2) st ^= 1;
  }
  constexpr int NQ = Tile::NQ;
  const int64_t sb = f.slot_base[s];
#pragma unroll
  for (int ta = 0; ta < NQ; ++ta)
#pragma unroll
    for (int tb = 0; tb < NQ; ++tb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = r0 + wr * 16 * NQ + ta * 16 + 4 * r + lane / 16;
        const int c = c0 + wc * 16 * NQ + tb * 16 + lane % 16;
        if (i >= m || c >= ncols) continue;
        const double v = t.acc[ta][tb][r];
        if (i < w)
          Y[(size_t)(a + i) * ncols + c] = v;
        else
          U[(size_t)(sb + i - w) * ncols + c] = v;
      }
}

// backward: X_s rows r0..r0+RT-1 = B_s^T [Y_s; -X_(R_s below the diagonal block)]
// (K = rows of B_s from r0 on: inv(L_ss) is lower triangular), staged as in
// the forward kernel.
// With nsplit > 1 block z takes a share of the K chunks and writes its
// partial tile to `part` (summed by k_bwd_reduce); launched with RT = 64.
template <int RT>
__global__ void __launch_bounds__(kBlock)
k_bwd_gemm(CholDev f, int t0, int ncols, int cbp, int ntile, const double* __restrict__ Y,
           double* __restrict__ X, int nsplit, double* __restrict__ part) {
  using Tile = MfmaTile<RT, bwd_kc(RT)>;
  constexpr int CT = RT, LDB = Tile::LDB;
  constexpr int KC = Tile::KC, LDA = Tile::LDA;
  constexpr int PER_T = RT * KC / kBlock;
  __shared__ double As[kStages][RT * LDA];
  __shared__ double Bs[kStages][KC * LDB];
  __shared__ int rows[RIDX];  // ancestor row indices of this block's K range
  const ColBlock cbk = col_block(cbp, ntile);  // u = row tile, v = split
  if (cbk.ct * CT >= ncols) return;           // padding tile: whole block
  int half;
  const int task = tile_task<RT>(t0, cbk.u, half);
  const int s = f.task_w_sn[task], r0 = f.task_w_r0[task] + RT * half;
  const int a = f.sn_start[s], w = f.sn_start[s + 1] - a;
  if (r0 >= w) return;  // whole block
  const int c0 = cbk.ct * CT;
  const int rb0 = f.sn_rowptr[s], m = f.sn_rowptr[s + 1] - rb0;
  const double* Br = f.brow + f.sn_valptr[s];
  const int tid = threadIdx.x, lane = tid % 64, wv = tid / 64;
  const int wr = wv / 2, wc = wv % 2;
  double ra[PER_T], rb[PER_T];
  // split-K: this block's share of the K chunks (all of them when nsplit == 1)
  const int nch = (m - r0 + KC - 1) / KC;
  const int per = (nch + nsplit - 1) / nsplit;
  const int kb = r0 + cbk.v * per * KC;
  const int ke = min(m, kb + per * KC);
  // The loads of a chunk are unconditional (indices clamped to elements
  // that exist) and nothing uses their values until they are staged after
  // the current chunk's products: the zeros past the edges and the sign of
  // the ancestor rows are applied then.  (Applied at the load, behind its
  // bounds test, they made every chunk wait on its loads before multiplying.)
  // per staged element u, four bits from bit 4u: A in range (1), B in range
  // (4), B from an ancestor row (8)
  static_assert(PER_T <= 8, "four flag bits per staged element");
  uint32_t keep = 0;
  auto load = [&](int i0) {
    keep = 0;
#pragma unroll
    for (int u = 0; u < PER_T; ++u) {
      const int e = tid + u * kBlock;
      // B operand first: its row index (from LDS, or from memory past the
      // cached range) is waited for before any load of the chunk is issued
      const int i2 = e / CT, cc = e % CT;
      const int ib = i0 + i2, c = c0 + cc;
      const bool bv = ib < m && c < ncols;
      const int ibc = min(ib, m - 1);
      const bool anc = ibc >= w;
      int ri = a + ibc;
      if (anc) ri = ibc - kb < RIDX ? rows[ibc - kb] : f.rowidx[rb0 + ibc];
      rb[u] = (anc ? X : Y)[(size_t)ri * ncols + min(c, ncols - 1)];
      // A operand: As[tt][ii] = B_s[i0 + ii][r0 + tt] (transposed while staging)
      const int ii = e / RT, tt = e % RT;
      const int i = i0 + ii, tc = r0 + tt;
      ra[u] = Br[(size_t)min(i, m - 1) * w + min(tc, w - 1)];
      const bool av = i < m && tc < w;
      keep |= ((av ? 1u : 0u) | (bv ? 4u : 0u) | (anc ? 8u : 0u)) << (4 * u);
    }
  };
  auto store = [&](int st) {
#pragma unroll
    for (int u = 0; u < PER_T; ++u) {
      const int e = tid + u * kBlock;
      const uint32_t kf = keep >> (4 * u);
      As[st][(e % RT) * LDA + e / RT] = (kf & 1u) ? ra[u] : 0.0;
      Bs[st][(e / CT) * LDB + e % CT] = (kf & 4u) ? ((kf & 8u) ? -rb[u] : rb[u]) : 0.0;
    }
  };
  Tile t;
  t.zero();
  for (int i = kb + threadIdx.x; i < min(ke, kb + RIDX); i += kBlock) rows[i - kb] = f.rowidx[rb0 + i];
  __syncthreads();
  int st = 0;
  if (kb < ke) {
    load(kb);
    store(0);
  }
  __syncthreads();
  for (int i0 = kb; i0 < ke; i0 += KC) {
    const bool more = i0 + KC < ke;
    if (more) load(i0 + KC);
    t.step(As[st], Bs[st], wr, wc, lane);
    if (more) {
      if (kStages == 1) __syncthreads();  // every wave has read the stage
      store(kStages == 1 ? 0 : st ^ 1);
    }
    __syncthreads();
    if (kStages == 2) st ^= 1;
  }
  constexpr int NQ = Tile::NQ;
#pragma unroll
  for (int ta = 0; ta < NQ; ++ta)
#pragma unroll
    for (int tb = 0; tb < NQ; ++tb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int lr = wr * 16 * NQ + ta * 16 + 4 * r + lane / 16;  // row within the tile
        const int tr = r0 + lr;
        const int c = c0 + wc * 16 * NQ + tb * 16 + lane % 16;
        if (tr >= w || c >= ncols) continue;
        const double v = t.acc[ta][tb][r];
        if (nsplit == 1) {
          X[(size_t)(a + tr) * ncols + c] = v;
        } else {
          part[(((size_t)cbk.v * ntile + cbk.u) * RT + lr) * ncols + c] = v;
        }
      }
}

constexpr int kMaxSplit = 16;  // split-K blocks per backward tile at most

// sums the split-K partials of one level in split order (deterministic)
__global__ void __launch_bounds__(kBlock)
k_bwd_reduce(CholDev f, int t0, int ntasks, int ncols, int cbp, int nsplit,
             const double* __restrict__ part, double* __restrict__ X) {
  const ColBlock cbk = col_block(cbp, 4);  // u = quarter, v = task
  const int tidx = cbk.v;
  const int task = t0 + tidx;
  const int s = f.task_w_sn[task], r0 = f.task_w_r0[task];
  const int a = f.sn_start[s], w = f.sn_start[s + 1] - a;
  const int c0 = cbk.ct * CTG;
  constexpr int RQ = RTK / 4;  // rows per block (the block order picks the quarter)
#pragma unroll
  for (int u = 0; u < RQ * CTG / kBlock; ++u) {
    const int e = threadIdx.x + u * kBlock;
    const int lr = cbk.u * RQ + e / CTG, c = c0 + e % CTG;
    const int tr = r0 + lr;
    if (tr >= w || c >= ncols) continue;
    // every partial in flight at once, then added in split order (the
    // zeros beyond nsplit leave the sum unchanged)
    double pv[kMaxSplit];
#pragma unroll
    for (int q = 0; q < kMaxSplit; ++q)
      pv[q] = q < nsplit ? part[(((size_t)q * ntasks + tidx) * RTK + lr) * ncols + c] : 0.0;
    double v = 0.0;
#pragma unroll
    for (int q = 0; q < kMaxSplit; ++q) v += pv[q];
    X[(size_t)(a + tr) * ncols + c] = v;
  }
}

// split factor of a backward level: enough blocks to occupy the chip (or
// the share of it the caller names)
int bwd_split(int ntw, int cb, int target = 2048) {
  const int blocks = ntw * cb;
  if (blocks >= target) return 1;
  return std::min(kMaxSplit, (target + blocks - 1) / blocks);
}

}  // namespace

size_t chol_split_bytes(const CholDev& f, int32_t ncols) {
  const int cb = (ncols + CTG - 1) / CTG;
  size_t need = 0;
  for (int lv = 0; lv < f.nlevels; ++lv) {
    const int ntw = f.level_w_host[lv + 1] - f.level_w_host[lv];
    const int ns = bwd_split(ntw, cb);
    if (ns > 1) need = std::max(need, (size_t)ns * ntw * RTK * ncols * sizeof(double));
  }
  return need;
}

// Tile size of a forward level: 64 x 64 output tiles, or 32 x 32 (four times
// the blocks, each with a quarter of the critical-path work) when the
// 64-tiles would not fill 512 blocks.  A backward level uses 32 x 32 tiles
// when none of its supernodes is wider than 32 (64-row tiles would be half
// padding); the others keep 64 x 64 tiles and split their longer K ranges
// (all rows of B_s) over blocks: measured on the torus 128 x 128 factor, 32 x
// 32 tiles there leave each block a long chain of load-bound chunks.
constexpr int kSmallLevelBlocks = 512;

void launch_chol_solve(hipStream_t s, const CholDev& f, int32_t ncols, const double* r, double* z,
                       double* W, double* Y, double* U, double* part, int32_t split_target) {
  double* X = z;  // rows by position: the solution block is the output
  dim3 blk(kBlock);
  const int cb = (ncols + CTG - 1) / CTG, cbp = pad_xcd(cb);
  const int cb32 = (ncols + 31) / 32, cbp32 = pad_xcd(cb32);
  for (int lv = 0; lv < f.nlevels; ++lv) {
    const int tw0 = f.level_w_host[lv], ntw = f.level_w_host[lv + 1] - tw0;
    const int tm0 = f.level_m_host[lv], ntm = f.level_m_host[lv + 1] - tm0;
    // the leaves (level 0) receive no updates: their rows of W are those of r
    const double* Wl = r;
    if (lv > 0) {
      prof::begin(s, DMC_KERNEL_CHOL_FWD_GATHER);
      hipLaunchKernelGGL(k_fwd_gather, dim3(cbp * GQ * ntw), blk, 0, s, f, tw0, ncols, cbp, r, U,
                         W);
      prof::end(s, DMC_KERNEL_CHOL_FWD_GATHER);
      Wl = W;
    }
    prof::begin(s, DMC_KERNEL_CHOL_FWD_SOLVE);
    if (ntm * cb < kSmallLevelBlocks)
      hipLaunchKernelGGL(k_fwd_gemm<32>, dim3(cbp32 * 2 * ntm), blk, 0, s, f, tm0, ncols, cbp32,
                         2 * ntm, Wl, Y, U);
    else
      hipLaunchKernelGGL(k_fwd_gemm<64>, dim3(cbp * ntm), blk, 0, s, f, tm0, ncols, cbp, ntm, Wl,
                         Y, U);
    prof::end(s, DMC_KERNEL_CHOL_FWD_SOLVE);
  }
  for (int lv = f.nlevels - 1; lv >= 0; --lv) {
    const int tw0 = f.level_w_host[lv], ntw = f.level_w_host[lv + 1] - tw0;
    prof::begin(s, DMC_KERNEL_CHOL_BWD_SOLVE);
    if (f.level_maxw_host[lv] <= 32) {
      // every supernode of the level is at most 32 wide (the dissection's
      // leaves and the lowest separators): 64-row tiles would be half padding
      hipLaunchKernelGGL(k_bwd_gemm<32>, dim3(cbp32 * 2 * ntw), blk, 0, s, f, tw0, ncols, cbp32,
                         2 * ntw, Y, X, 1, (double*)nullptr);
    } else {
      const int ns = part ? bwd_split(ntw, cb, std::min<int>(split_target, 2048)) : 1;
      hipLaunchKernelGGL(k_bwd_gemm<64>, dim3(cbp * ntw * ns), blk, 0, s, f, tw0, ncols, cbp, ntw,
                         Y, X, ns, part);
      if (ns > 1)
        hipLaunchKernelGGL(k_bwd_reduce, dim3(cbp * 4 * ntw), blk, 0, s, f, tw0, ntw, ncols, cbp,
                           ns, part, X);
    }
    prof::end(s, DMC_KERNEL_CHOL_BWD_SOLVE);
  }
}

}  // namespace dmc
