// Internal declarations shared by the host driver and the kernel files.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/dmc.h"
#include "profile.h"

namespace dmc {

constexpr int kBlock = 256;
// XCDs of an MI355X: the dispatcher deals consecutive workgroups of a launch
// to them in turn (workgroup b runs on XCD b mod 8), each with its own L2.
constexpr int kXcds = 8;
// Entries past the end of the device copies of M's column and value arrays
// (column 0, value 0), so a kernel may read the first entries of a row's
// pattern without testing them against the row's end.
constexpr int kMatPad = 32;

// An empty asm statement that takes v as an operand (no instruction is
// emitted): the load that produced v must have been issued before it, so a
// group of loads followed by their pins stays in flight together, where the
// compiler would otherwise move each load behind the bounds test that
// selects its value and wait on them one by one.
__device__ __forceinline__ void pin(double& v) { asm volatile("" : "+v"(v)); }

inline int pad_xcd(int blocks) { return (blocks + kXcds - 1) / kXcds * kXcds; }
constexpr size_t kAlign = 256;

inline size_t align_up(size_t x, size_t a = kAlign) { return (x + a - 1) / a * a; }

// First word of every window record ("DMC2" in memory order).
constexpr int32_t kRecordMagic = 0x32434d44;

// Header words of a record (int32 each, 128 bytes in all; see dmc.h).
enum RecordHeader {
  kHdrMagic = 0, kHdrT, kHdrK, kHdrN, kHdrNc, kHdrCoefBits, kHdrAnchorBits, kHdrDictBits,
  kHdrPrecision, kHdrDictMode, kHdrHasDiff, kHdrUsedLo, kHdrUsedHi, kHdrDictWords,
  kHdrStepLo, kHdrStepHi, kHeaderBytes = 128
};

// One entry of a record's dictionary-column or coefficient-row table: the
// range of the coded values (float32), the bit width (low byte) and, for a
// dictionary column, its mode (second byte: 0 values, 1 difference from the
// previous window's column), and the first 32-bit word of its segment in the
// record's variable part.
struct SegEntry {
  float lo, hi;
  uint32_t bits_mode;
  uint32_t word_off;
};

// 32-bit words of a segment of `count` codes of `bits` bits (bits = 0: raw
// values of `real` bytes), rounded up to an even count (8-byte boundary).
__host__ __device__ inline uint32_t seg_words(uint32_t count, uint32_t bits, uint32_t real) {
  const uint64_t w = bits ? ((uint64_t)count * bits + 31) / 32 : ((uint64_t)count * real + 3) / 4;
  return (uint32_t)(w + (w & 1));
}

// code j of a packed segment (bit j b of the segment's bit string, least
// significant bit first; b <= 16); the second word is read only when the
// code reaches into it
__device__ inline uint32_t get_code(const uint32_t* __restrict__ seg, uint32_t j, uint32_t bits) {
  const uint64_t pos = (uint64_t)j * bits;
  const uint32_t w = (uint32_t)(pos >> 5), sh = (uint32_t)(pos & 31);
  uint64_t v = seg[w];
  if (sh + bits > 32) v |= (uint64_t)seg[w + 1] << 32;
  return (uint32_t)(v >> sh) & ((1u << bits) - 1u);
}

// Byte layout of one window record (see dmc.h).  The fixed part holds the
// header, the dictionary-column table [3][k], the coefficient-row table
// [3][k], the anchor ranges [3] and the anchor segments [3]; the variable
// part (from off_var) holds the dictionary segments and then the coefficient
// rows, packed back to back at the offsets the tables give.  `bytes` is the
// capacity: every segment at its widest (dict_bits, coef_bits).
struct RecordLayout {
  int32_t T = 0, k = 0, n = 0, nc = 0;
  int32_t coef_bits = 0, anchor_bits = 0, dict_bits = 0, precision = 0;
  int32_t dict_mode = 0;
  double coef_step = 0.0;
  size_t real = 8;            // bytes per raw value
  size_t off_dtab = 0, off_rtab = 0, off_arange = 0, off_anchors = 0, anchor_seg = 0;
  size_t off_var = 0;
  size_t bytes = 0;
};

RecordLayout record_layout(int32_t n, int32_t T, int32_t k, int32_t nc, const dmc_params& p);

// Device-side supernodal Cholesky factor of the normal matrix (built on the
// host by build_cholesky, see chol_host.h).
struct CholDev {
  int32_t n = 0, ns = 0, nlevels = 0;
  const int32_t* perm = nullptr;        // elimination position -> vertex (host solve only:
                                        // the device solves work in positions)
  const int32_t* sn_start = nullptr;    // [ns+1]
  const int32_t* sn_rowptr = nullptr;   // [ns+1]
  const int32_t* rowidx = nullptr;
  const int64_t* sn_valptr = nullptr;   // offsets of B_s (m_s x w_s)
  const double* brow = nullptr;         // B_s row-major
  const int64_t* slot_base = nullptr;   // [ns+1] update slots of each supernode
  const int32_t* contrib_ptr = nullptr; // [n+1] per column: update slots aimed at it
  const int32_t* contrib_slot = nullptr;
  // work items (supernode, first row of a 64-row tile), grouped by level:
  // tiles over the w_s columns of each supernode, and over its m_s rows
  const int32_t* task_w_sn = nullptr;
  const int32_t* task_w_r0 = nullptr;
  const int32_t* task_m_sn = nullptr;
  const int32_t* task_m_r0 = nullptr;
  const int32_t* level_w_host = nullptr;  // host arrays [nlevels + 1]
  const int32_t* level_m_host = nullptr;
  const int32_t* level_maxw_host = nullptr;  // host [nlevels]: widest supernode of a level
  int64_t nslots = 0;
};

// Symbolic structure of the factor on the device, for the numeric
// factorisation at mesh creation (kernels_factor.hip): supernode blocks L_s
// (m_s x w_s row-major at sn_valptr[s]), their row indices, the supernode of
// every column, the lower triangle of P M P^T by column, and each target's
// update segments (chol_host.h).
struct FactorDev {
  int32_t n = 0;
  const int32_t* sn_start = nullptr;
  const int32_t* sn_rowptr = nullptr;
  const int32_t* rowidx = nullptr;
  const int32_t* sn_of = nullptr;
  const int64_t* sn_valptr = nullptr;
  const int32_t* acol_ptr = nullptr;
  const int32_t* acol_row = nullptr;
  const double* acol_val = nullptr;
  const int32_t* seg_ptr = nullptr;
  const int32_t* seg_d = nullptr;
  const int32_t* seg_p1 = nullptr;
  const int32_t* seg_p2 = nullptr;
  double* L = nullptr;     // the factor's blocks (work, zeroed before the launch)
  double* B = nullptr;     // the solve operators B_s, row-major (output)
  int32_t* fail = nullptr; // smallest supernode with a non-positive pivot + 1 (init INT_MAX)
};
// Work lists of the numeric factorisation, by level (offsets on the host,
// lists on the device): update tiles (target, row tile << 16 | column tile),
// the level's supernodes and their largest block, operator tasks (supernode,
// first of 64 rows) for all supernodes.
struct FactorPlan {
  int32_t nlevels = 0;
  const int32_t* tile_off = nullptr;  // host [nlevels + 1]
  const int32_t* tile_sn = nullptr;   // device
  const int32_t* tile_rc = nullptr;   // device
  const int32_t* sn_off = nullptr;    // host [nlevels + 1]
  const int32_t* lv_sn = nullptr;     // device
  const int32_t* maxm = nullptr;      // host [nlevels]: tallest block of the level
  const int32_t* maxw = nullptr;      // host [nlevels]: widest block of the level
  const int32_t* op_sn = nullptr;     // device
  const int32_t* op_row = nullptr;    // device
  int32_t op_off_total = 0;
};
void launch_factor_numeric(hipStream_t s, const FactorDev& f, const FactorPlan& p);
// out[r] = in[map[r]] for n rows of ncols doubles
void launch_permute_rows(hipStream_t s, const double* in, const int32_t* map, int32_t n,
                         int32_t ncols, double* out);

// Device-side mesh data.
struct MeshDev {
  int32_t n = 0, nnz = 0, nc = 0, laplacian = 0;
  int32_t m_nnz = 0;
  const int32_t* rowptr = nullptr;   // [n+1]  CSR of the adjacency C
  const int32_t* col = nullptr;      // [nnz]
  const double* w64 = nullptr;       // [n] 1/d_i (uniform) or d_i (combinatorial)
  const float* w32 = nullptr;
  const int32_t* anchors = nullptr;  // [nc]
  // The decoder's n-row blocks (right-hand sides, CG vectors, solutions, the
  // anchor response) hold vertex perm[p] in row p, perm the factor's
  // elimination order: ring members sit a few rows apart (nested dissection
  // keeps each subdomain contiguous), so the sparse products find their
  // neighbour rows in the L2, and the supernodal solves read and write their
  // rows in place.  The operators below are indexed by that row position.
  const int32_t* dpos = nullptr;     // [n] vertex -> row position
  const int32_t* d_rowptr = nullptr; // [n+1] C by position (entries in each vertex's ring order)
  const int32_t* d_col = nullptr;    // [nnz] positions of the ring members
  const double* d_w64 = nullptr;     // [n] w64 by position
  const int32_t* d_slot = nullptr;   // [n] anchor slot of a position, or -1
  const int32_t* d_anchors = nullptr;// [nc] row position of each anchor
  const int32_t* m_rowptr = nullptr; // [n+1] CSR of L^T L + I_N^T I_N, by position
  const int32_t* m_col = nullptr;
  const double* m_val = nullptr;
  const double* m_dinv = nullptr;    // [n] 1 / diagonal, by position
  CholDev chol;
  // anchor response G = (L^T L + I_N^T I_N)^{-1} I_N^T, [n][nc], row p for
  // vertex perm[p] (nullptr when not built: the decoder then solves 3T
  // columns per window)
  const double* G = nullptr;
  double G_resid = 0.0;  // largest relative residual of G's columns
  double solve_entries = 0.0;  // entries of the solve operators (one triangular solve)
};

// Per-window stats written by the kernels (device).
struct StatsDev {
  int32_t sweeps[3];
  int32_t shifts[3];
  double resid[3];
};

// ---- kernel launchers (kernels_*.hip) --------------------------------------

// Delta coordinates for F frames; fpb frames per workgroup (a tuning knob).
void launch_delta(hipStream_t s, const MeshDev& m, const void* in, void* out, int32_t F,
                  int32_t precision, int fpb = 8);

// Autocorrelation of nw consecutive windows of T frames each:
// frames [nw*T][n][3] -> R [nw][3][T][T] float64.  `part` is scratch of
// autocorr_scratch_bytes(...) bytes.  P = vertex blocks per window (a tuning
// knob; 0 = the default for n and nw).
size_t autocorr_scratch_bytes(int32_t n, int32_t T, int32_t nw, int32_t precision, int P = 0);
void launch_autocorr(hipStream_t s, const void* frames, int32_t n, int32_t T, int32_t nw,
                     int32_t precision, void* part, double* R, int P = 0);
int autocorr_blocks(int n, int nw);

// Orthogonal iterations + Ritz + dictionary quantisation over a chain of nw
// windows of T frames (window w starts from window w-1's U_k).
struct OiArgs {
  const double* R;       // [nw][3][T][T]
  int32_t nw, T, k;
  int32_t precision;
  int32_t init;          // DMC_INIT_*
  int32_t ncoord;        // blocks per window: 3 (x, y, z), or 1 for independent blocks
  const void* q_start;   // per init: [3][T][k], [nw][3][T][k] or Omega [T][k] (real)
  const float* q_learned;  // DMC_INIT_LEARNED: [nw][ncoord][T][k] predicted starts
  void* u_out;           // [nw][ncoord][T][k] real (may be nullptr)
  double* u_canon;       // [nw][ncoord][T][k] float64 canonical U (or nullptr)
  int32_t max_sweeps;
  double tol;
  StatsDev* stats;       // [nw]
  // chained path (DMC_INIT_PREV): scratch for the deferred Ritz step,
  // [nw][ncoord][T*k + k*k] float64 (Q, then H = Q^T R Q) and [nw][ncoord]
  // flags, or nullptr (the Ritz step then runs inside the chain)
  double* ritz_qh;
  int32_t* ritz_flag;
};
void launch_oi(hipStream_t s, const OiArgs& a);
// jobs[b] = (index into args, first window, end window, coordinate); the
// (TMAX, KR) class is the largest T (<= 32 or <= 64) and k (<= 16 or <= 32)
// of the jobs
void launch_oi_batch(hipStream_t s, int tmax, int kr, int precision, const OiArgs* args,
                     const int4* jobs, int njobs);
// the launchers of one (TMAX, KR) class (TMAX 32 or 64, KR 16 or 32), each
// instantiated in a unit of its own
template <int TMAX, int KR>
void launch_oi_t(hipStream_t st, const OiArgs& a);
template <int TMAX, int KR>
void launch_oi_batch_t(hipStream_t st, int precision, const OiArgs* args, const int4* jobs,
                       int njobs);

// Learned start (row-wise perceptron on the sketch R Omega).
int mlp_param_count(int k);
int mlp_bwd_parts();
void launch_mlp_sketch(hipStream_t s, const double* R, int nb, int T, const double* omega, float* S);
void launch_mlp_forward(hipStream_t s, const float* theta, int k, const float* S, int N, float* Q,
                        float* cache);
void launch_mlp_loss(hipStream_t s, const float* Q, const double* U, int T, int k, int nb, double mu,
                     float* dQ, double* loss);
void launch_mlp_backward(hipStream_t s, const float* theta, int k, const float* S, int N,
                         const float* cache, const float* dQ, float* dZ, float* partial,
                         float* grad);
void launch_mlp_adam(hipStream_t s, float* theta, const float* grad, float* m, float* v, int count,
                     int step, double lr, double b1, double b2, double eps);

// Projection (Eq. 9) of the delta coordinates (Eq. 3-4, formed on the fly
// from the frames [nw*T][n][3], never stored) + per-row ranges +
// quantisation (Eq. 10) for nw windows.
// The coefficient rows go into the records packed at the bits of their
// row table (k_row_table, after the dictionary segments).
size_t project_scratch_bytes(int32_t n, int32_t T, int32_t k, int32_t nw, int32_t precision);
void launch_project_quantise(hipStream_t s, const MeshDev& m, const void* frames, int32_t T,
                             int32_t k, int32_t nw, int32_t precision, const double* u_tilde,
                             uint8_t* records, size_t rec_bytes, const RecordLayout& lay,
                             void* scratch, void* coef_out);

// Anchor values of nw windows (Eq. 12): gather + quantisation into records;
// part: anchors_scratch_bytes(nw) bytes.
size_t anchors_scratch_bytes(int32_t nw);
void launch_anchors(hipStream_t s, const MeshDev& m, const void* frames, int32_t T, int32_t nw,
                    int32_t precision, uint8_t* records, size_t rec_bytes, const RecordLayout& lay,
                    double* part);

// Dictionary of nw windows from their canonical U (u_canon [nw][3][T][k]
// float64): column table, packed segments and header words of each record,
// and the dequantised dictionary u_tilde [nw][3][T][k] the projection uses.
void launch_dict_code(hipStream_t s, const double* u_canon, int32_t nw, const RecordLayout& lay,
                      uint8_t* records, size_t rec_bytes, double* u_tilde);
// zeros after each record's used bytes (run last)
void launch_zero_tail(hipStream_t s, uint8_t* records, int32_t nw, size_t rec_bytes);

// headers of nw records rec_bytes apart (and the zeros of their alignment gaps)
void launch_write_headers(hipStream_t s, uint8_t* records, int32_t nw, size_t rec_bytes,
                          const RecordLayout& lay);

// ---- decode ----------------------------------------------------------------

// Right-hand side of the normal equations for every window of a sequence,
// columns j = 3*t + c for global frame t.  B0 and b are [n][ncols] float64.
struct SeqLayout {
  int32_t nw_full, T;        // full windows
  int32_t T_tail;            // 0 if none
  RecordLayout full, tail;
  size_t rec_bytes_full;
};
// The dequantised dictionaries of every window, ut [window][3][T][k]
// (dict_decode_doubles(sl) doubles), which the decode kernels below read.
size_t dict_decode_doubles(const SeqLayout& sl);
void launch_dict_decode(hipStream_t s, const uint8_t* records, const SeqLayout& sl, double* ut);
// Temporal-subspace decode (X_wc = Z_wc U~_wc^T + G A^_wc, Eq. 12 by linearity):
// columns of the reduced system (3k per window), dequantised coefficients
// Yd [n][nz], its right-hand side L^T Yd (no anchor term), the dense anchor
// values [nc][3F], the anchor response's right-hand sides I_N^T [n][nc], and
// the product that writes the frames [F][n][3] from Z [n][nz], G and A^.
int32_t reduced_cols(const SeqLayout& sl);
void launch_coef_rows(hipStream_t s, const MeshDev& m, const uint8_t* records,
                      const SeqLayout& sl, double* Yd);
void launch_rhs_reduced(hipStream_t s, const MeshDev& m, int32_t nz, const double* Yd, double* b,
                        double* bb);
void launch_anchor_values(hipStream_t s, const MeshDev& m, const uint8_t* records,
                          const SeqLayout& sl, double* Ah);
// Direct decode's right-hand side b [n][3F] = L^T (Y^ U~^T) + I_N^T A^ from
// the coefficient rows Yd [n][nz] (launch_coef_rows), the dictionaries ut and
// the dense anchor values Ah [nc][3F] (NULL: no anchor term); bb
// (optional): per-block partial b.b per column (the first half of the CG
// partials, [cg_part_rows(n)][3F]).
void launch_rhs_from_coefs(hipStream_t s, const MeshDev& m, const SeqLayout& sl,
                           const double* Yd, const double* ut, const double* Ah, double* b,
                           double* bb);
void launch_anchor_unit_rhs(hipStream_t s, const MeshDev& m, double* b);
// Reference norms of the reduced columns (after launch_cg_init, with b the
// reduced right-hand side): the test on them bounds every frame's full-system
// relative residual by tol.  gram_part: group_gram_doubles(n, sl) doubles.
size_t group_gram_doubles(int32_t n, const SeqLayout& sl);
void launch_group_ref(hipStream_t s, const MeshDev& m, const uint8_t* records, const SeqLayout& sl,
                      const double* ut, const double* b, const double* Ah, double tol,
                      double* gram_part, double* bnorm2);
void launch_compose(hipStream_t s, const MeshDev& m, const uint8_t* records, const SeqLayout& sl,
                    const double* ut, const double* Z, const double* Ah, int32_t precision,
                    void* frames_out);

struct CgBuffers {
  double *x, *r, *p, *q;
  double *z, *W, *Y, *U;  // preconditioned residual and triangular-solve work
  double* S;                    // split-K partials of the backward solve
  // blocks a backward level is split up to (fewer where other work runs
  // beside the solve, as in the batched form's graph branches)
  int32_t split_target = 2048;
  double* part;      // [nblk_rows][ncols] x 2
  double *rz, *rr, *bnorm2, *alpha, *beta;
  int32_t* done;     // [ncols]
  double* resid;     // [ncols]
};
size_t cg_part_rows(int32_t n);
// zero_x: set x = 0 (needed only when no iteration will run: the first
// step_a, with first set, writes x = alpha p)
// bb_done: the right-hand side's b.b partials are already in cb.part
void launch_cg_init(hipStream_t s, const MeshDev& m, int32_t ncols, const double* b,
                    const CgBuffers& cb, int32_t precond, bool zero_x, bool bb_done = false);
// one iteration = step_a (q = M p, alpha, x and r updates, residual check)
// then, unless every column has converged, step_b (preconditioner, beta, p);
// first: the first iteration after launch_cg_init (x taken as zero)
void launch_cg_step_a(hipStream_t s, const MeshDev& m, int32_t ncols, const CgBuffers& cb,
                      int32_t precond, double tol, bool first);
void launch_cg_step_b(hipStream_t s, const MeshDev& m, int32_t ncols, const CgBuffers& cb,
                      int32_t precond);
// Cholesky-preconditioned solve started from the preconditioner's own
// solution: launch_cg_norms reduces the b.b partials the right-hand side
// left in cb.part (bnorm2, done = 0, resid = 1); launch_cg_warm_start sets
// x = (L L^T)^-1 b (r still holds b), forms the residual norms of
// b - M x without storing it and marks the columns within tol;
// launch_cg_restart then (for columns still open) writes r = b - M x, the
// first search direction p = (L L^T)^-1 r and rz, after which
// launch_cg_step_a (first = false) and launch_cg_step_b continue.
void launch_cg_norms(hipStream_t s, const MeshDev& m, int32_t ncols, const CgBuffers& cb);
void launch_cg_warm_start(hipStream_t s, const MeshDev& m, int32_t ncols, const CgBuffers& cb,
                          double tol);
void launch_cg_restart(hipStream_t s, const MeshDev& m, int32_t ncols, const CgBuffers& cb);
// summary of a solve on the device: out[0] = max relative residual, out[1] =
// 1.0 if every column converged
void launch_cg_summary(hipStream_t s, const CgBuffers& cb, int32_t ncols, double* out);
// part: split-K scratch of chol_split_bytes(f, ncols) bytes (nullptr: no split)
size_t chol_split_bytes(const CholDev& f, int32_t ncols);
// z = (L L^T)^-1 r for ncols columns (rows by position; z also serves the
// backward solve as its solution block); split_target: blocks a backward
// level is split up to (at most 2048)
void launch_chol_solve(hipStream_t s, const CholDev& f, int32_t ncols, const double* r, double* z,
                       double* W, double* Y, double* U, double* part,
                       int32_t split_target = 2048);
void launch_precond_apply(hipStream_t s, const MeshDev& m, int32_t ncols, const CgBuffers& cb,
                          double* p_out);
// X [n][3F] (rows by position) -> frames [F][n][3] (vertex order)
void launch_to_frames(hipStream_t s, const MeshDev& m, const double* X, int32_t F,
                      int32_t precision, void* frames_out);

}  // namespace dmc
