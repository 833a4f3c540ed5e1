// C ABI entry points: argument validation, context/mesh lifetime, scratch
// management and the order of launches for encode and decode.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <array>
#include <chrono>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "chol_host.h"
#include "dmc_internal.h"
#include "mesh_host.h"

// Scratch of dmc_encode_window_noalloc: a fixed device array instead of
// allocated memory (the delta coordinates, the chain's pieces and the
// window's stats of one encode).  Every GPU the library runs on holds its own
// copy, at its own address, until the process ends.  In host code the name is
// only a stand-in: kernels and copies take the address hipGetSymbolAddress
// returned for the device (noalloc_scratch below), never the name itself.
constexpr size_t kNoAllocScratchBytes = DMC_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_scratch[kMaxDevices] = {};  // per device, set by dmc_create
}  // namespace

struct dmc_ctx_s {
  int device = 0;
  hipStream_t stream = nullptr;
  void* scratch = nullptr;
  size_t scratch_bytes = 0;
  bool scratch_external = false;  // caller's workspace (dmc_set_workspace): never freed or grown
  void* pinned = nullptr;  // host staging for stats and convergence flags
  size_t pinned_bytes = 0;
  void* stats = nullptr;   // per-window device stats (kept apart from scratch)
  size_t stats_bytes = 0;
  hipEvent_t ev[3] = {nullptr, nullptr, nullptr};  // encode / decode timers of the stats
  std::vector<dmc_mesh_s*> meshes;
  // learned start registered by dmc_learned_start (caller-owned device memory)
  int32_t learned_T = 0, learned_k = 0;
  const double* learned_omega = nullptr;
  const float* learned_theta = nullptr;
};

struct dmc_mesh_s {
  dmc_ctx ctx = nullptr;
  dmc::MeshDev dev;
  std::vector<void*> allocations;
  std::vector<int32_t> level_w, level_m;  // host copies of the factor's level -> task ranges
  std::vector<int32_t> level_maxw;        // widest supernode of each level
  double factor_info[DMC_FACTOR_INFO_LEN] = {};
  int32_t g_iters = 0;  // CG iterations of the anchor response (0: not built)
};

namespace {

thread_local std::string g_error;

dmc_status fail(dmc_status st, const std::string& msg) {
  g_error = msg;
  return st;
}

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t _e = (expr);                                                             \
    if (_e != hipSuccess)                                                               \
      return fail(DMC_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(_e));  \
  } while (0)

dmc_status check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(DMC_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
  return DMC_OK;
}

// Scratch carving: a bump allocator over the context's scratch buffer.
struct Carve {
  std::vector<size_t> sizes;
  size_t add(size_t bytes) {
    sizes.push_back(dmc::align_up(std::max<size_t>(bytes, 1)));
    size_t off = 0;
    for (size_t i = 0; i + 1 < sizes.size(); ++i) off += sizes[i];
    return off;
  }
  size_t total() const {
    size_t t = 0;
    for (size_t s : sizes) t += s;
    return t;
  }
};

dmc_status ensure_scratch(dmc_ctx ctx, size_t bytes) {
  if (bytes <= ctx->scratch_bytes) return DMC_OK;
  if (ctx->scratch_external)
    return fail(DMC_ERR_BUFFER_TOO_SMALL, "the workspace holds " +
                                              std::to_string(ctx->scratch_bytes) + " bytes, the call needs " +
                                              std::to_string(bytes) + " (dmc_workspace_bytes)");
  if (ctx->scratch) {
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    HIP_TRY(hipFree(ctx->scratch));
    ctx->scratch = nullptr;
    ctx->scratch_bytes = 0;
  }
  const size_t want = dmc::align_up(bytes, size_t(1) << 20);
  if (hipMalloc(&ctx->scratch, want) != hipSuccess) {
    ctx->scratch = nullptr;
    (void)hipGetLastError();
    return fail(DMC_ERR_OUT_OF_MEMORY, "cannot allocate " + std::to_string(want) + " scratch bytes");
  }
  ctx->scratch_bytes = want;
  return DMC_OK;
}

// The stats and staging buffers are allocated with the context at sizes that
// cover thousands of windows; they grow only beyond that, and never while the
// caller's workspace is in use (those calls must not allocate).
constexpr size_t kStatsBytes = size_t(256) << 10;
constexpr size_t kPinnedBytes = size_t(1) << 20;

dmc_status ensure_stats(dmc_ctx ctx, size_t bytes) {
  if (bytes <= ctx->stats_bytes) return DMC_OK;
  if (ctx->scratch_external)
    return fail(DMC_ERR_BUFFER_TOO_SMALL, "too many windows for the context's stats buffer");
  if (ctx->stats) {
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    HIP_TRY(hipFree(ctx->stats));
  }
  ctx->stats = nullptr;
  ctx->stats_bytes = 0;
  const size_t want = std::max<size_t>(bytes, 4096);
  if (hipMalloc(&ctx->stats, want) != hipSuccess) {
    ctx->stats = nullptr;
    (void)hipGetLastError();
    return fail(DMC_ERR_OUT_OF_MEMORY, "cannot allocate stats buffer");
  }
  ctx->stats_bytes = want;
  return DMC_OK;
}

dmc_status ensure_pinned(dmc_ctx ctx, size_t bytes) {
  if (bytes <= ctx->pinned_bytes) return DMC_OK;
  if (ctx->scratch_external)
    return fail(DMC_ERR_BUFFER_TOO_SMALL, "too many columns for the context's staging buffer");
  if (ctx->pinned) {
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    HIP_TRY(hipHostFree(ctx->pinned));
  }
  ctx->pinned = nullptr;
  ctx->pinned_bytes = 0;
  const size_t want = std::max<size_t>(bytes, 1 << 16);
  HIP_TRY(hipHostMalloc(&ctx->pinned, want, hipHostMallocDefault));
  ctx->pinned_bytes = want;
  return DMC_OK;
}

dmc_status check_params(const dmc_params* p, int32_t T, bool for_decode = false) {
  if (!p) return fail(DMC_ERR_INVALID_ARG, "params is NULL");
  if (T < 1 || T > 64) return fail(DMC_ERR_INVALID_ARG, "window length T must be in 1..64");
  if (p->k < 1 || p->k > 32) return fail(DMC_ERR_INVALID_ARG, "k must be in 1..32");
  if (p->precision != DMC_FP64 && p->precision != DMC_FP32 && p->precision != DMC_BF16)
    return fail(DMC_ERR_INVALID_ARG, "precision must be DMC_FP64, DMC_FP32 or DMC_BF16");
  for (int32_t b : {p->coef_bits, p->anchor_bits, p->dict_bits})
    if (b < 0 || b > 16) return fail(DMC_ERR_INVALID_ARG, "bits must be in 0..16");
  if (p->dict_mode != DMC_DICT_PLAIN && p->dict_mode != DMC_DICT_ADAPTIVE)
    return fail(DMC_ERR_INVALID_ARG, "dict_mode must be DMC_DICT_PLAIN or DMC_DICT_ADAPTIVE");
  if (p->dict_mode == DMC_DICT_ADAPTIVE && p->dict_bits < 1)
    return fail(DMC_ERR_INVALID_ARG, "DMC_DICT_ADAPTIVE needs dict_bits >= 1");
  if (!(p->coef_step >= 0.0) || !std::isfinite(p->coef_step))
    return fail(DMC_ERR_INVALID_ARG, "coef_step must be finite and >= 0");
  if (p->coef_step > 0.0 && p->coef_bits < 1)
    return fail(DMC_ERR_INVALID_ARG, "coef_step needs coef_bits >= 1 (the widest row)");
  if (!for_decode) {
    if (p->init < DMC_INIT_PREV || p->init > DMC_INIT_LEARNED)
      return fail(DMC_ERR_INVALID_ARG, "unknown init");
    if (p->oi_max_sweeps < 1) return fail(DMC_ERR_INVALID_ARG, "oi_max_sweeps must be >= 1");
    // the precision form needs a sweep with bfloat16 products and at least
    // one full-precision refinement sweep before the Ritz step
    if (p->precision == DMC_BF16 && p->oi_max_sweeps < 2)
      return fail(DMC_ERR_INVALID_ARG, "DMC_BF16 needs oi_max_sweeps >= 2");
    if (!(p->oi_tol >= 0.0)) return fail(DMC_ERR_INVALID_ARG, "oi_tol must be >= 0");
  }
  if (p->cg_max_iters < 1) return fail(DMC_ERR_INVALID_ARG, "cg_max_iters must be >= 1");
  if (!(p->cg_tol >= 0.0)) return fail(DMC_ERR_INVALID_ARG, "cg_tol must be >= 0");
  if (p->precond < DMC_PRECOND_NONE || p->precond > DMC_PRECOND_CHOLESKY)
    return fail(DMC_ERR_INVALID_ARG, "unknown preconditioner");
  return DMC_OK;
}

size_t real_size(int32_t precision) { return precision == DMC_FP64 ? 8 : 4; }

// Bits per vertex per frame and coordinate of one window's record (Eq. 13
// read per coordinate), from a host copy of its header and tables: q counts
// the coefficient rows' segments and their table entries, q_a the anchor
// segments and ranges, q_d the dictionary columns' segments and table
// entries, q_s the record's used bytes (header and alignment included).
void record_bpvf(const dmc::RecordLayout& l, const uint8_t* head, double out[4]) {
  const double vf = 3.0 * l.n * l.T;
  const uint32_t rl = (uint32_t)l.real;
  const dmc::SegEntry* dt = (const dmc::SegEntry*)(head + l.off_dtab);
  const dmc::SegEntry* rt = (const dmc::SegEntry*)(head + l.off_rtab);
  double q = 0.0, qd = 0.0;
  for (int e = 0; e < 3 * l.k; ++e) {
    q += 32.0 * dmc::seg_words((uint32_t)l.n, rt[e].bits_mode & 0xffu, rl) + 8.0 * sizeof(dmc::SegEntry);
    qd += 32.0 * dmc::seg_words((uint32_t)l.T, dt[e].bits_mode & 0xffu, rl) + 8.0 * sizeof(dmc::SegEntry);
  }
  const double qa = 3.0 * (8.0 * l.anchor_seg + 64.0);
  const int32_t* h = (const int32_t*)head;
  const uint64_t used = (uint64_t)(uint32_t)h[dmc::kHdrUsedLo] |
                        ((uint64_t)(uint32_t)h[dmc::kHdrUsedHi] << 32);
  out[0] = q / vf;
  out[1] = qa / vf;
  out[2] = qd / vf;
  out[3] = 8.0 * (double)used / vf;
}

// Host copies of the header and tables (the first off_arange + 24 bytes) of
// nw_full records of layout `full` at records + w * full.bytes and, if
// `tail` is given, of one more record after them; synchronises the stream.
dmc_status read_record_heads(dmc_ctx ctx, const uint8_t* records, int32_t nw_full,
                             const dmc::RecordLayout& full, const dmc::RecordLayout* tail,
                             std::vector<std::vector<uint8_t>>& heads) {
  const size_t hf = full.off_arange + 24, ht = tail ? tail->off_arange + 24 : 0;
  dmc_status st = ensure_pinned(ctx, (size_t)nw_full * hf + ht);
  if (st != DMC_OK) return st;
  uint8_t* h = (uint8_t*)ctx->pinned;
  if (nw_full)
    HIP_TRY(hipMemcpy2DAsync(h, hf, records, full.bytes, hf, nw_full, hipMemcpyDeviceToHost,
                             ctx->stream));
  if (tail)
    HIP_TRY(hipMemcpyAsync(h + (size_t)nw_full * hf, records + (size_t)nw_full * full.bytes, ht,
                           hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  heads.clear();
  for (int32_t w = 0; w < nw_full; ++w) heads.emplace_back(h + w * hf, h + (w + 1) * hf);
  if (tail) heads.emplace_back(h + (size_t)nw_full * hf, h + (size_t)nw_full * hf + ht);
  return DMC_OK;
}

void fill_bits(dmc_window_stats* st, const dmc::RecordLayout& l, const uint8_t* head) {
  double b[4];
  record_bpvf(l, head, b);
  st->q = b[0];
  st->q_a = b[1];
  st->q_d = b[2];
  st->q_s = b[3];
}

void fill_stats(dmc_window_stats* st, const dmc::StatsDev& s, const dmc::RecordLayout& l,
                const uint8_t* head) {
  st->T = l.T;
  st->k = l.k;
  for (int c = 0; c < 3; ++c) {
    st->oi_sweeps[c] = s.sweeps[c];
    st->oi_resid[c] = s.resid[c];
    st->chol_shifts[c] = s.shifts[c];
  }
  fill_bits(st, l, head);
}

// Algorithm 1 did not reach oi_tol for some coordinate of some window (its
// iterations ran and ended above the tolerance, at the sweep cap or where
// the precision form's refinement stopped improving); an exact start (no
// sweeps) is not an iteration.
bool oi_not_converged(const dmc::StatsDev* s, int32_t nw, double tol) {
  for (int32_t w = 0; w < nw; ++w)
    for (int c = 0; c < 3; ++c)
      if (s[w].sweeps[c] > 0 && !(s[w].resid[c] <= tol)) return true;
  return false;
}

float elapsed_ms(hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.f;
  return ms;
}

// Encode nw windows of length T starting at frames (one chain).
dmc_status encode_chain(dmc_ctx ctx, const dmc::MeshDev& m, const void* frames, int32_t T,
                        int32_t nw, int32_t k, const dmc_params& p, const void* q_start,
                        uint8_t* records, const dmc::RecordLayout& lay, void* u_out,
                        void* coef_out, uint8_t* ws,
                        dmc::StatsDev* stats_dev) {
  hipStream_t s = ctx->stream;
  // scratch pieces (chain_scratch_bytes counts them in this order)
  uint8_t* cur = ws;
  double* R = (double*)cur;
  cur += dmc::align_up((size_t)nw * 3 * T * T * 8);
  void* part = cur;
  cur += dmc::align_up(dmc::autocorr_scratch_bytes(m.n, T, nw, p.precision));
  double* u_canon = (double*)cur;
  cur += dmc::align_up((size_t)nw * 3 * T * k * 8);
  double* u_tilde = (double*)cur;
  cur += dmc::align_up((size_t)nw * 3 * T * k * 8);
  double* apart = (double*)cur;
  cur += dmc::anchors_scratch_bytes(nw);
  float* sk = nullptr;
  float* ql = nullptr;
  if (p.init == DMC_INIT_LEARNED) {
    sk = (float*)cur;
    cur += dmc::align_up((size_t)nw * 3 * T * 32 * 4);
    ql = (float*)cur;
    cur += dmc::align_up((size_t)nw * 3 * T * k * 4);
  }
  // the chained start defers each window's Ritz step to one parallel pass
  double* ritz_qh = nullptr;
  int32_t* ritz_flag = nullptr;
  if (p.init == DMC_INIT_PREV) {
    ritz_qh = (double*)cur;
    cur += dmc::align_up((size_t)nw * 3 * (T * k + k * k) * 8);
    ritz_flag = (int32_t*)cur;
    cur += dmc::align_up((size_t)nw * 3 * 4);
  }
  void* proj = cur;
  dmc::launch_write_headers(s, records, nw, lay.bytes, lay);
  dmc::launch_autocorr(s, frames, m.n, T, nw, p.precision, part, R);
  if (p.init == DMC_INIT_LEARNED) {
    dmc::launch_mlp_sketch(s, R, nw * 3, T, ctx->learned_omega, sk);
    dmc::launch_mlp_forward(s, ctx->learned_theta, k, sk, nw * 3 * T, ql, nullptr);
  }
  dmc::OiArgs oa{};
  oa.R = R;
  oa.nw = nw;
  oa.T = T;
  oa.k = k;
  oa.precision = p.precision;
  oa.init = p.init;
  oa.ncoord = 3;
  oa.q_start = p.init == DMC_INIT_EXACT ? nullptr : q_start;
  oa.q_learned = ql;
  oa.u_out = u_out;
  oa.u_canon = u_canon;
  oa.max_sweeps = p.oi_max_sweeps;
  oa.tol = p.oi_tol;
  oa.stats = stats_dev;
  oa.ritz_qh = ritz_qh;
  oa.ritz_flag = ritz_flag;
  dmc::launch_oi(s, oa);
  dmc::launch_dict_code(s, u_canon, nw, lay, records, lay.bytes, u_tilde);
  dmc::launch_project_quantise(s, m, frames, T, k, nw, p.precision, u_tilde, records, lay.bytes,
                               lay, proj, coef_out);
  dmc::launch_anchors(s, m, frames, T, nw, p.precision, records, lay.bytes, lay, apart);
  dmc::launch_zero_tail(s, records, nw, lay.bytes);
  return check_launch("encode kernels");
}

size_t chain_scratch_bytes(int32_t n, int32_t T, int32_t nw, int32_t k, int32_t precision,
                           int32_t init) {
  const size_t learned = init == DMC_INIT_LEARNED
                             ? dmc::align_up((size_t)nw * 3 * T * 32 * 4) +
                                   dmc::align_up((size_t)nw * 3 * T * k * 4)
                             : 0;
  const size_t ritz = init == DMC_INIT_PREV
                          ? dmc::align_up((size_t)nw * 3 * (T * k + k * k) * 8) +
                                dmc::align_up((size_t)nw * 3 * 4)
                          : 0;
  return dmc::align_up((size_t)nw * 3 * T * T * 8) +
         dmc::align_up(dmc::autocorr_scratch_bytes(n, T, nw, precision)) +
         2 * dmc::align_up((size_t)nw * 3 * T * k * 8) + dmc::anchors_scratch_bytes(nw) +
         learned + ritz + dmc::align_up(dmc::project_scratch_bytes(n, T, k, nw, precision));
}

// The learned start needs a network registered for this window length and k.
dmc_status check_learned(dmc_ctx ctx, const dmc_params& p, int32_t T) {
  if (p.init != DMC_INIT_LEARNED) return DMC_OK;
  if (!ctx->learned_theta || !ctx->learned_omega)
    return fail(DMC_ERR_INVALID_ARG, "DMC_INIT_LEARNED needs dmc_learned_start first");
  if (ctx->learned_T != T || ctx->learned_k != std::min(p.k, T))
    return fail(DMC_ERR_INVALID_ARG, "the registered learned start is for another T or k");
  return DMC_OK;
}

// Decoder buffers for ncols right-hand sides, carved from one region.
struct DecodeLayout {
  size_t o_x, o_r, o_p, o_q, o_part, o_small, o_z, o_W, o_Y, o_U, o_S, o_Ah, o_gram, o_ut,
      total;
};

// ah_values, gram_values: doubles of the dense anchor values [nc][3F] and of
// the partial Gram matrices of the reduced decode (0 for the full decode,
// whose anchor values follow b)
// ut_values: doubles of the decoded dictionaries
DecodeLayout decode_layout(const dmc::MeshDev& m, int32_t ncols, bool chol,
                           size_t ah_values = 0, size_t gram_values = 0, size_t ut_values = 0) {
  const size_t vec = (size_t)m.n * ncols * 8;
  const size_t nrb = dmc::cg_part_rows(m.n);
  Carve cv;
  DecodeLayout d{};
  d.o_x = cv.add(vec);
  d.o_r = cv.add(vec + (size_t)m.nc * ncols * 8);  // b, then r; anchor values after
  d.o_p = cv.add(vec);
  d.o_q = cv.add(vec);                             // back-projection, then q
  d.o_part = cv.add(2 * nrb * ncols * 8);
  d.o_small = cv.add((size_t)ncols * 8 * 6 + (size_t)ncols * 4);
  if (chol) {
    d.o_z = cv.add(vec);
    d.o_W = cv.add(vec);
    d.o_Y = cv.add(vec);
    d.o_U = cv.add((size_t)m.chol.nslots * ncols * 8);
    d.o_S = cv.add(dmc::chol_split_bytes(m.chol, ncols));
  }
  d.o_Ah = cv.add(ah_values * 8);
  d.o_gram = cv.add(gram_values * 8);
  d.o_ut = cv.add(ut_values * 8);
  d.total = cv.total();
  return d;
}

// Cost weights of the decode forms, per column of the solve and per output
// column: a solved column costs about 4 flops per solve-operator entry (the
// forward and backward solves), weighted 4x because the level-scheduled solve
// runs at about a quarter of the efficiency of the dense anchor product, which
// costs 2 n n_c flops per output column.
inline double solve_cost_per_column(const dmc::MeshDev& m) { return 16.0 * m.solve_entries; }
inline double anchor_cost_per_column(const dmc::MeshDev& m) { return 2.0 * m.n * (double)m.nc; }

// How a sequence is decoded: the temporal-subspace form (solve the 3k columns
// L^T Y^^T of each window, then X = Z U~^T + G A^) when the mesh holds its
// anchor response and nz S + 3F A < 3F S (S, A the costs above, nz the
// reduced columns); otherwise the direct form (3T columns per window).
struct DecodePlan {
  bool reduced = false;
  int32_t F = 0, ncols = 0;  // frames; columns of the solve
  DecodeLayout lay{};
};

DecodePlan decode_plan(const dmc::MeshDev& m, const dmc::SeqLayout& sl, const dmc_params& p) {
  DecodePlan d;
  d.F = sl.nw_full * sl.T + sl.T_tail;
  const int32_t nz = dmc::reduced_cols(sl);
  const double S = solve_cost_per_column(m), A = anchor_cost_per_column(m);
  d.reduced = m.G != nullptr && nz < 3 * d.F &&
              (double)nz * S + 3.0 * d.F * A < 3.0 * d.F * S;
  d.ncols = d.reduced ? nz : 3 * d.F;
  d.lay = decode_layout(m, d.ncols, p.precond == DMC_PRECOND_CHOLESKY,
                        d.reduced ? (size_t)m.nc * 3 * d.F : 0,
                        d.reduced ? dmc::group_gram_doubles(m.n, sl) : 0,
                        dmc::dict_decode_doubles(sl));
  return d;
}

dmc::CgBuffers decode_buffers(uint8_t* ws, const DecodeLayout& d, int32_t ncols, bool chol) {
  dmc::CgBuffers cb;
  cb.x = (double*)(ws + d.o_x);
  cb.r = (double*)(ws + d.o_r);
  cb.p = (double*)(ws + d.o_p);
  cb.q = (double*)(ws + d.o_q);
  cb.part = (double*)(ws + d.o_part);
  cb.z = chol ? (double*)(ws + d.o_z) : nullptr;
  cb.W = chol ? (double*)(ws + d.o_W) : nullptr;
  cb.Y = chol ? (double*)(ws + d.o_Y) : nullptr;
  cb.U = chol ? (double*)(ws + d.o_U) : nullptr;
  cb.S = chol ? (double*)(ws + d.o_S) : nullptr;
  double* small = (double*)(ws + d.o_small);
  cb.rz = small;
  cb.rr = small + ncols;
  cb.bnorm2 = small + 2 * ncols;
  cb.alpha = small + 3 * ncols;
  cb.beta = small + 4 * ncols;
  cb.resid = small + 5 * ncols;
  cb.done = (int32_t*)(small + 6 * ncols);
  return cb;
}

// Decode with a fixed number of conjugate-gradient iterations and no host
// synchronisation (capturable); summary[0..1] receives the largest relative
// residual and whether every column converged.
void decode_enqueue_setup(hipStream_t s, const dmc::MeshDev& m, const uint8_t* records,
                          const dmc::SeqLayout& sl, const dmc_params& p, const DecodePlan& d,
                          const dmc::CgBuffers& cb, uint8_t* ws, bool zero_x) {
  double* Ah = (double*)(ws + d.lay.o_Ah);
  double* ut = (double*)(ws + d.lay.o_ut);
  // the windows' dictionaries (in order: a column may be coded as the
  // difference from the previous window's)
  dmc::launch_dict_decode(s, records, sl, ut);
  // the right-hand side kernel also forms the b.b partials the Cholesky
  // start needs (the init kernel then has nothing left to do)
  double* bb = p.precond == DMC_PRECOND_CHOLESKY ? cb.part : nullptr;
  if (d.reduced) {
    dmc::launch_coef_rows(s, m, records, sl, cb.q);
    dmc::launch_rhs_reduced(s, m, d.ncols, cb.q, cb.r, bb);
    dmc::launch_anchor_values(s, m, records, sl, Ah);
  } else {
    // b = L^T (Y^ U~^T) formed as (L^T Y^) U~^T: the dequantised coefficient
    // rows (in q), the anchor values after b, then the expansion
    double* Ah = cb.r + (size_t)m.n * d.ncols;
    dmc::launch_coef_rows(s, m, records, sl, cb.q);
    dmc::launch_anchor_values(s, m, records, sl, Ah);
    dmc::launch_rhs_from_coefs(s, m, sl, cb.q, ut, m.nc ? Ah : nullptr, cb.r, bb);
  }
  if (p.precond == DMC_PRECOND_CHOLESKY)
    dmc::launch_cg_norms(s, m, d.ncols, cb);  // the solve starts from the factor's solution
  else
    dmc::launch_cg_init(s, m, d.ncols, cb.r, cb, p.precond, zero_x, bb != nullptr);
  // the test on the reduced columns bounds every frame's full-system residual
  // (r still holds b here)
  if (d.reduced)
    dmc::launch_group_ref(s, m, records, sl, ut, cb.r, Ah, p.cg_tol,
                          (double*)(ws + d.lay.o_gram), cb.bnorm2);
}

void decode_enqueue_finish(hipStream_t s, const dmc::MeshDev& m, const uint8_t* records,
                           const dmc::SeqLayout& sl, const dmc_params& p, const DecodePlan& d,
                           const dmc::CgBuffers& cb, const uint8_t* ws, void* frames_out) {
  if (d.reduced)
    dmc::launch_compose(s, m, records, sl, (const double*)(ws + d.lay.o_ut), cb.x,
                        (const double*)(ws + d.lay.o_Ah), p.precision, frames_out);
  else
    dmc::launch_to_frames(s, m, cb.x, d.F, p.precision, frames_out);
}

void decode_enqueue_fixed(hipStream_t s, const dmc::MeshDev& m, const uint8_t* records,
                          const dmc::SeqLayout& sl, const dmc_params& p, const DecodePlan& d,
                          uint8_t* ws, void* frames_out, int iters, double* summary,
                          int32_t split_target = 2048) {
  const bool chol = p.precond == DMC_PRECOND_CHOLESKY;
  dmc::CgBuffers cb = decode_buffers(ws, d.lay, d.ncols, chol);
  cb.split_target = split_target;
  decode_enqueue_setup(s, m, records, sl, p, d, cb, ws, iters < 1);
  if (p.precond == DMC_PRECOND_CHOLESKY) {
    // iteration 1 is the start from the factor's solution; the later ones
    // continue the preconditioned iterations from it (converged columns stay)
    dmc::launch_cg_warm_start(s, m, d.ncols, cb, p.cg_tol);
    for (int it = 2; it <= iters; ++it) {
      if (it == 2)
        dmc::launch_cg_restart(s, m, d.ncols, cb);
      else
        dmc::launch_cg_step_b(s, m, d.ncols, cb, p.precond);
      dmc::launch_cg_step_a(s, m, d.ncols, cb, p.precond, p.cg_tol, false);
    }
  } else {
    for (int it = 1; it <= iters; ++it) {
      dmc::launch_cg_step_a(s, m, d.ncols, cb, p.precond, p.cg_tol, it == 1);
      if (it < iters) dmc::launch_cg_step_b(s, m, d.ncols, cb, p.precond);
    }
  }
  dmc::launch_cg_summary(s, cb, d.ncols, summary);
  decode_enqueue_finish(s, m, records, sl, p, d, cb, ws, frames_out);
}

// Conjugate-gradient iterations on the system launch_cg_init set up, with a
// host check of convergence every check_every iterations (every iteration
// with the Cholesky preconditioner, which converges in one or two).
dmc_status cg_iterate(dmc_ctx ctx, const dmc::MeshDev& m, int32_t ncols,
                      const dmc::CgBuffers& cb, int32_t precond, double tol, int32_t max_iters,
                      int32_t* iters_out, bool* all_done_out) {
  hipStream_t s = ctx->stream;
  dmc_status st = ensure_pinned(ctx, (size_t)ncols * 12 + 4096);
  if (st != DMC_OK) return st;
  int32_t* h_done = (int32_t*)ctx->pinned;
  const int check_every = precond == DMC_PRECOND_CHOLESKY ? 1 : 16;
  int it = 0;
  bool all_done = false;
  while (it < max_iters) {
    dmc::launch_cg_step_a(s, m, ncols, cb, precond, tol, it == 0);
    ++it;
    if (it % check_every == 0 || it == max_iters) {
      st = check_launch("cg kernels");
      if (st != DMC_OK) return st;
      HIP_TRY(hipMemcpyAsync(h_done, cb.done, (size_t)ncols * 4, hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      all_done = true;
      for (int j = 0; j < ncols; ++j) all_done = all_done && h_done[j];
      if (all_done || it == max_iters) break;
    }
    dmc::launch_cg_step_b(s, m, ncols, cb, precond);
  }
  *iters_out = it;
  *all_done_out = all_done;
  return DMC_OK;
}

// Decode every window of a sequence in one solve over 3F columns.
dmc_status decode_all(dmc_ctx ctx, const dmc::MeshDev& m, const uint8_t* records,
                      const dmc::SeqLayout& sl, const dmc_params& p, void* frames_out,
                      int32_t* iters_out, double* resid_out) {
  hipStream_t s = ctx->stream;
  const DecodePlan d = decode_plan(m, sl, p);
  const int32_t ncols = d.ncols;
  const bool chol = p.precond == DMC_PRECOND_CHOLESKY;
  dmc_status st = ensure_scratch(ctx, d.lay.total);
  if (st != DMC_OK) return st;
  st = ensure_pinned(ctx, (size_t)ncols * 12 + 4096);
  if (st != DMC_OK) return st;
  uint8_t* ws = (uint8_t*)ctx->scratch;
  const dmc::CgBuffers cb = decode_buffers(ws, d.lay, ncols, chol);

  decode_enqueue_setup(s, m, records, sl, p, d, cb, ws, p.cg_max_iters < 1);
  st = check_launch("decode setup kernels");
  if (st != DMC_OK) return st;
  int32_t* h_done = (int32_t*)ctx->pinned;
  double* h_res = (double*)((uint8_t*)ctx->pinned + dmc::align_up((size_t)ncols * 4));
  int32_t it = 0;
  bool all_done = false;
  if (chol && p.cg_max_iters >= 1) {
    // The solve starts from the Cholesky factor's own solution x = (L L^T)^-1
    // b, whose residual is checked without being stored (the factor is exact
    // up to rounding, so that start nearly always meets the tolerance).  The
    // frames are formed right after that check and the host reads the
    // convergence flags once, at the end; columns that have not converged
    // continue with preconditioned iterations from the start and the frames
    // are formed again.
    auto read_flags = [&]() -> dmc_status {
      HIP_TRY(hipMemcpyAsync(h_done, cb.done, (size_t)ncols * 4, hipMemcpyDeviceToHost, s));
      HIP_TRY(hipMemcpyAsync(h_res, cb.resid, (size_t)ncols * 8, hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      all_done = true;
      for (int j = 0; j < ncols; ++j) all_done = all_done && h_done[j];
      return DMC_OK;
    };
    dmc::launch_cg_warm_start(s, m, ncols, cb, p.cg_tol);
    it = 1;
    decode_enqueue_finish(s, m, records, sl, p, d, cb, ws, frames_out);
    st = check_launch("cg kernels and frames");
    if (st != DMC_OK) return st;
    st = read_flags();
    if (st != DMC_OK) return st;
    if (!all_done && it < p.cg_max_iters) {
      dmc::launch_cg_restart(s, m, ncols, cb);
      while (!all_done && it < p.cg_max_iters) {
        if (it > 1) dmc::launch_cg_step_b(s, m, ncols, cb, p.precond);
        dmc::launch_cg_step_a(s, m, ncols, cb, p.precond, p.cg_tol, false);
        ++it;
        st = check_launch("cg kernels");
        if (st != DMC_OK) return st;
        st = read_flags();
        if (st != DMC_OK) return st;
      }
      decode_enqueue_finish(s, m, records, sl, p, d, cb, ws, frames_out);
      st = check_launch("frames");
      if (st != DMC_OK) return st;
      HIP_TRY(hipStreamSynchronize(s));
    }
  } else {
    st = cg_iterate(ctx, m, ncols, cb, p.precond, p.cg_tol, p.cg_max_iters, &it, &all_done);
    if (st != DMC_OK) return st;
    decode_enqueue_finish(s, m, records, sl, p, d, cb, ws, frames_out);
    st = check_launch("frames");
    if (st != DMC_OK) return st;
    HIP_TRY(hipMemcpyAsync(h_res, cb.resid, (size_t)ncols * 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  double rmax = 0.0;
  for (int j = 0; j < ncols; ++j) rmax = std::max(rmax, h_res[j]);
  if (iters_out) *iters_out = it;
  if (resid_out) *resid_out = rmax;
  if (!all_done)
    return fail(DMC_ERR_NOT_CONVERGED, "conjugate gradients stopped at cg_max_iters with max "
                                       "relative residual " + std::to_string(rmax));
  return DMC_OK;
}

// Everything dmc_mesh_create computes on the host: adjacency (Eq. 2),
// validation, the normal matrix of Eq. (12) and its Cholesky factor.  Parts
// of at most kNdLeaf vertices end the nested dissection: larger leaves mean
// fewer tree levels (each level is a few dependent launches of the solve)
// for somewhat more operator entries in the dense leaf blocks.
constexpr int32_t kNdLeaf = 128;

// numeric: also factorise on the host (else only the ordering and symbolic
// analysis run here, and dmc_mesh_create factorises on the device)
dmc_status build_mesh_host(int32_t n, int32_t n_tris, const int32_t* tris, int32_t n_anchors,
                           const int32_t* anchors, int32_t laplacian, dmc::HostCsr& C,
                           dmc::HostCsr& M, dmc::CholFactor& F, double info[DMC_FACTOR_INFO_LEN],
                           bool numeric) {
  if (n < 1 || n_tris < 1 || !tris) return fail(DMC_ERR_INVALID_ARG, "need n >= 1 and triangles");
  if (laplacian != DMC_LAP_UNIFORM && laplacian != DMC_LAP_COMBINATORIAL)
    return fail(DMC_ERR_INVALID_ARG, "unknown Laplacian");
  if (n_anchors < 0 || (n_anchors > 0 && !anchors))
    return fail(DMC_ERR_INVALID_ARG, "bad anchor array");
  std::vector<char> seen(n, 0);
  for (int32_t a = 0; a < n_anchors; ++a) {
    if (anchors[a] < 0 || anchors[a] >= n)
      return fail(DMC_ERR_INVALID_ARG, "anchor index out of range");
    if (seen[anchors[a]]) return fail(DMC_ERR_INVALID_ARG, "repeated anchor index");
    seen[anchors[a]] = 1;
  }
  std::string msg;
  if (!dmc::build_adjacency(n, n_tris, tris, C, msg)) return fail(DMC_ERR_INVALID_ARG, msg);
  for (int32_t i = 0; i < n; ++i)
    if (C.rowptr[i + 1] == C.rowptr[i])
      return fail(DMC_ERR_INVALID_ARG, "vertex " + std::to_string(i) +
                                           " has no neighbour (Eq. 3 undefined)");
  const int32_t missing = dmc::unanchored_components(C, anchors, n_anchors);
  if (missing > 0)
    return fail(DMC_ERR_SINGULAR, std::to_string(missing) +
                                      " connected component(s) without an anchor: the "
                                      "anchored system is singular");
  dmc::build_normal_matrix(C, laplacian, anchors, n_anchors, M);
  const auto t0 = std::chrono::steady_clock::now();
  if (!dmc::build_cholesky_symbolic(M, kNdLeaf, F, msg, &C)) return fail(DMC_ERR_SINGULAR, msg);
  if (numeric && !dmc::factor_numeric_host(F, msg)) return fail(DMC_ERR_SINGULAR, msg);
  const double secs =
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  info[0] = (double)F.sn_valptr[F.nsuper];
  info[1] = (double)F.nnz_exact;
  info[2] = F.nsuper;
  info[3] = F.nlevels;
  info[4] = F.flops;
  info[5] = secs;
  // entries of the solve operators one triangular solve reads (lower
  // triangle of inv(L_ss) plus the dense L_os inv(L_ss)), and update rows
  double entries = 0.0, updates = 0.0, leaf_rows = 0.0;
  for (int32_t s = 0; s < F.nsuper; ++s) {
    const double w = F.sn_start[s + 1] - F.sn_start[s];
    const double m = F.sn_rowptr[s + 1] - F.sn_rowptr[s];
    entries += w * (w + 1) / 2 + (m - w) * w;
    updates += m - w;
    if (F.sn_level[s] == 0) leaf_rows += w;
  }
  info[6] = entries;
  info[7] = updates;
  info[8] = leaf_rows;
  return DMC_OK;
}

}  // namespace

namespace dmc {

RecordLayout record_layout(int32_t n, int32_t T, int32_t k, int32_t nc, const dmc_params& p) {
  RecordLayout l;
  l.T = T;
  l.k = k;
  l.n = n;
  l.nc = nc;
  l.coef_bits = p.coef_bits;
  l.anchor_bits = p.anchor_bits;
  l.dict_bits = p.dict_bits;
  l.precision = p.precision;
  l.dict_mode = p.dict_mode;
  l.coef_step = p.coef_bits > 0 ? p.coef_step : 0.0;
  l.real = real_size(p.precision);
  const uint32_t rl = (uint32_t)l.real;
  l.off_dtab = kHeaderBytes;
  l.off_rtab = l.off_dtab + (size_t)3 * k * sizeof(SegEntry);
  l.off_arange = l.off_rtab + (size_t)3 * k * sizeof(SegEntry);
  l.off_anchors = align_up(l.off_arange + 3 * 8);
  l.anchor_seg = 4 * (size_t)seg_words((uint32_t)(T * nc), (uint32_t)p.anchor_bits, rl);
  l.off_var = align_up(l.off_anchors + 3 * l.anchor_seg);
  // every segment at its widest
  l.bytes = align_up(l.off_var + 4 * (size_t)3 * k *
                                     (seg_words((uint32_t)T, (uint32_t)p.dict_bits, rl) +
                                      seg_words((uint32_t)n, (uint32_t)p.coef_bits, rl)));
  return l;
}

}  // namespace dmc

// The anchor response G = (L^T L + I_N^T I_N)^{-1} I_N^T of a mesh (one column
// per anchor), solved on the device by conjugate gradients with the Cholesky
// preconditioner, aiming at a relative residual of kAnchorResponseTol in at
// most kAnchorResponseIters iterations.  It lets the decoder solve 3k instead
// of 3T columns per window (its residual enters the decoder's test).  It is
// left unbuilt (the direct decode is used) when its product costs more than
// half a solved column even at k = T / 2 (2 A > S), when it would take more
// than kAnchorResponseBytes, when its allocation fails or when its largest
// residual is above kAnchorResponseAccept.
constexpr double kAnchorResponseTol = 1e-14;
constexpr double kAnchorResponseAccept = 1e-12;
constexpr int32_t kAnchorResponseIters = 8;
constexpr size_t kAnchorResponseBytes = size_t(2) << 30;

dmc_status build_anchor_response(dmc_ctx ctx, dmc_mesh m) {
  dmc::MeshDev& dv = m->dev;
  const int32_t nc = dv.nc;
  const size_t bytes = (size_t)dv.n * nc * 8;
  if (nc < 1 || bytes > kAnchorResponseBytes) return DMC_OK;
  if (2.0 * anchor_cost_per_column(dv) > solve_cost_per_column(dv)) return DMC_OK;
  const DecodeLayout dl = decode_layout(dv, nc, true);
  // mesh set-up solves in a temporary buffer of its own (the context's
  // scratch may be a caller's workspace sized for encode and decode)
  uint8_t* ws = nullptr;
  if (hipMalloc(&ws, dl.total) != hipSuccess) {
    (void)hipGetLastError();
    return DMC_OK;  // no anchor response: the decoder uses the direct form
  }
  struct Release {
    uint8_t* p;
    hipStream_t s;
    ~Release() {
      (void)hipStreamSynchronize(s);
      (void)hipFree(p);
    }
  } release{ws, ctx->stream};
  dmc_status st = DMC_OK;
  const dmc::CgBuffers cb = decode_buffers(ws, dl, nc, true);
  hipStream_t s = ctx->stream;
  dmc::launch_anchor_unit_rhs(s, dv, cb.r);
  dmc::launch_cg_init(s, dv, nc, cb.r, cb, DMC_PRECOND_CHOLESKY, kAnchorResponseIters < 1);
  st = check_launch("anchor response setup");
  if (st != DMC_OK) return st;
  int32_t it = 0;
  bool done = false;  // below kAnchorResponseTol everywhere (not required)
  st = cg_iterate(ctx, dv, nc, cb, DMC_PRECOND_CHOLESKY, kAnchorResponseTol, kAnchorResponseIters,
                  &it, &done);
  if (st != DMC_OK) return st;
  double* h_res = (double*)((uint8_t*)ctx->pinned + dmc::align_up((size_t)nc * 4));
  HIP_TRY(hipMemcpyAsync(h_res, cb.resid, (size_t)nc * 8, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  double rmax = 0.0;
  for (int32_t j = 0; j < nc; ++j) rmax = std::max(rmax, h_res[j]);
  if (!(rmax <= kAnchorResponseAccept)) return DMC_OK;
  void* G = nullptr;
  if (hipMalloc(&G, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return DMC_OK;
  }
  m->allocations.push_back(G);
  HIP_TRY(hipMemcpyAsync(G, cb.x, bytes, hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  dv.G = (const double*)G;
  dv.G_resid = rmax;
  m->g_iters = it;
  return DMC_OK;
}

extern "C" {

const char* dmc_last_error(void) { return g_error.c_str(); }

dmc_status dmc_create(int32_t device, void* hip_stream, dmc_ctx* out) {
  if (!out) return fail(DMC_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count == 0)
    return fail(DMC_ERR_DEVICE, "no HIP device");
  if (device < 0 || device >= count) return fail(DMC_ERR_INVALID_ARG, "device index out of range");
  HIP_TRY(hipSetDevice(device));
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, device));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(DMC_ERR_DEVICE, std::string("built for gfx950, device is ") + prop.gcnArchName);
  if (device >= kMaxDevices) return fail(DMC_ERR_UNSUPPORTED, "device index above 63");
  {
    // the device's address of the fixed scratch array, once per device,
    // with the device current
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_scratch[device]) {
      void* ptr = nullptr;
      const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !ptr)
        return fail(DMC_ERR_DEVICE,
                    std::string("hipGetSymbolAddress of the fixed scratch: ") + hipGetErrorString(e));
      g_noalloc_scratch[device] = ptr;
    }
  }
  dmc_ctx c = new dmc_ctx_s();
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  // the stats and staging buffers and the timers are made here, so that the
  // encode and decode calls themselves need no allocation
  bool ok = hipMalloc(&c->stats, kStatsBytes) == hipSuccess;
  if (ok) c->stats_bytes = kStatsBytes;
  ok = ok && hipHostMalloc(&c->pinned, kPinnedBytes, hipHostMallocDefault) == hipSuccess;
  if (ok) c->pinned_bytes = kPinnedBytes;
  for (int e = 0; e < 3 && ok; ++e) ok = hipEventCreate(&c->ev[e]) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    dmc_destroy(c);
    return fail(DMC_ERR_OUT_OF_MEMORY, "cannot allocate the context's stats and staging buffers");
  }
  *out = c;
  return DMC_OK;
}

void dmc_destroy(dmc_ctx ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  for (dmc_mesh_s* m : ctx->meshes) {
    for (void* p : m->allocations) (void)hipFree(p);
    delete m;
  }
  if (ctx->scratch && !ctx->scratch_external) (void)hipFree(ctx->scratch);
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  if (ctx->stats) (void)hipFree(ctx->stats);
  for (hipEvent_t e : ctx->ev)
    if (e) (void)hipEventDestroy(e);
  delete ctx;
}

dmc_status dmc_set_stream(dmc_ctx ctx, void* hip_stream) {
  if (!ctx) return fail(DMC_ERR_INVALID_ARG, "ctx is NULL");
  ctx->stream = (hipStream_t)hip_stream;
  return DMC_OK;
}

size_t dmc_scratch_bytes(dmc_ctx ctx) {
  return ctx && !ctx->scratch_external ? ctx->scratch_bytes : 0;
}

dmc_status dmc_set_workspace(dmc_ctx ctx, void* dev_ptr, size_t bytes) {
  if (!ctx) return fail(DMC_ERR_INVALID_ARG, "ctx is NULL");
  if ((dev_ptr == nullptr) != (bytes == 0))
    return fail(DMC_ERR_INVALID_ARG, "give both a workspace and its size, or neither");
  if (dev_ptr && (uintptr_t)dev_ptr % dmc::kAlign != 0)
    return fail(DMC_ERR_INVALID_ARG, "the workspace must be 256-byte aligned");
  HIP_TRY(hipSetDevice(ctx->device));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  if (ctx->scratch && !ctx->scratch_external) HIP_TRY(hipFree(ctx->scratch));
  ctx->scratch = dev_ptr;
  ctx->scratch_bytes = bytes;
  ctx->scratch_external = dev_ptr != nullptr;
  return DMC_OK;
}

// Numeric factorisation of the mesh's normal matrix on the device from the
// host's symbolic analysis F (kernels_factor.hip): uploads the structure and
// the work lists, runs the levels, keeps the solve operators B_s (the solve
// kernels' brow) and frees the rest.  DMC_ERR_SINGULAR if a pivot is not
// positive.
static dmc_status factor_on_device(dmc_ctx ctx, dmc_mesh m, const dmc::CholFactor& F) {
  hipStream_t s = ctx->stream;
  const int32_t n = F.n, ns = F.nsuper, nl = F.nlevels;
  // work lists: supernodes by level, update tiles (lower-triangle tiles of the
  // levels above the leaves), operator tasks
  std::vector<int32_t> sn_off(nl + 1, 0), lv_sn, tile_off(nl + 1, 0), tile_sn, tile_rc, maxm(nl, 0),
      maxw(nl, 0), op_sn, op_row, sn_of(n);
  std::vector<std::vector<int32_t>> by_level(nl);
  for (int32_t q = 0; q < ns; ++q) by_level[F.sn_level[q]].push_back(q);
  for (int32_t lv = 0; lv < nl; ++lv) {
    for (int32_t q : by_level[lv]) {
      const int32_t w = F.sn_start[q + 1] - F.sn_start[q];
      const int32_t mm = F.sn_rowptr[q + 1] - F.sn_rowptr[q];
      lv_sn.push_back(q);
      maxm[lv] = std::max(maxm[lv], mm);
      maxw[lv] = std::max(maxw[lv], w);
      if (F.seg_ptr[q + 1] > F.seg_ptr[q])
        for (int32_t cb = 0; cb * 64 < w; ++cb)
          for (int32_t rb = cb; rb * 64 < mm; ++rb) {
            tile_sn.push_back(q);
            tile_rc.push_back(rb << 16 | cb);
          }
    }
    sn_off[lv + 1] = (int32_t)lv_sn.size();
    tile_off[lv + 1] = (int32_t)tile_sn.size();
  }
  for (int32_t q = 0; q < ns; ++q) {
    for (int32_t j = F.sn_start[q]; j < F.sn_start[q + 1]; ++j) sn_of[j] = q;
    const int32_t mm = F.sn_rowptr[q + 1] - F.sn_rowptr[q];
    for (int32_t r0 = 0; r0 < mm; r0 += 64) {
      op_sn.push_back(q);
      op_row.push_back(r0);
    }
  }
  std::vector<void*> tmp;
  bool ok = true;
  auto dev = [&](const void* src, size_t bytes, bool keep) -> void* {
    void* d = nullptr;
    if (hipMalloc(&d, std::max<size_t>(bytes, 8)) != hipSuccess) {
      ok = false;
      return nullptr;
    }
    (keep ? m->allocations : tmp).push_back(d);
    if (src && bytes && hipMemcpy(d, src, bytes, hipMemcpyHostToDevice) != hipSuccess) ok = false;
    return d;
  };
  const dmc::CholDev& cd = m->dev.chol;
  const size_t vals = (size_t)F.sn_valptr[ns];
  dmc::FactorDev fd;
  fd.n = n;
  fd.sn_start = cd.sn_start;
  fd.sn_rowptr = cd.sn_rowptr;
  fd.rowidx = cd.rowidx;
  fd.sn_valptr = cd.sn_valptr;
  fd.sn_of = (const int32_t*)dev(sn_of.data(), sn_of.size() * 4, false);
  fd.acol_ptr = (const int32_t*)dev(F.acol_ptr.data(), F.acol_ptr.size() * 4, false);
  fd.acol_row = (const int32_t*)dev(F.acol_row.data(), F.acol_row.size() * 4, false);
  fd.acol_val = (const double*)dev(F.acol_val.data(), F.acol_val.size() * 8, false);
  fd.seg_ptr = (const int32_t*)dev(F.seg_ptr.data(), F.seg_ptr.size() * 4, false);
  fd.seg_d = (const int32_t*)dev(F.seg_d.data(), F.seg_d.size() * 4, false);
  fd.seg_p1 = (const int32_t*)dev(F.seg_p1.data(), F.seg_p1.size() * 4, false);
  fd.seg_p2 = (const int32_t*)dev(F.seg_p2.data(), F.seg_p2.size() * 4, false);
  fd.L = (double*)dev(nullptr, vals * 8, false);
  fd.B = (double*)dev(nullptr, vals * 8, true);
  const int32_t fail_init = INT32_MAX;
  fd.fail = (int32_t*)dev(&fail_init, 4, false);
  dmc::FactorPlan fp;
  fp.nlevels = nl;
  fp.tile_off = tile_off.data();
  fp.tile_sn = (const int32_t*)dev(tile_sn.data(), tile_sn.size() * 4, false);
  fp.tile_rc = (const int32_t*)dev(tile_rc.data(), tile_rc.size() * 4, false);
  fp.sn_off = sn_off.data();
  fp.lv_sn = (const int32_t*)dev(lv_sn.data(), lv_sn.size() * 4, false);
  fp.maxm = maxm.data();
  fp.maxw = maxw.data();
  fp.op_sn = (const int32_t*)dev(op_sn.data(), op_sn.size() * 4, false);
  fp.op_row = (const int32_t*)dev(op_row.data(), op_row.size() * 4, false);
  fp.op_off_total = (int32_t)op_sn.size();
  int32_t failed = INT32_MAX;
  if (ok && hipMemsetAsync(fd.L, 0, vals * 8, s) != hipSuccess) ok = false;
  if (ok) {
    dmc::launch_factor_numeric(s, fd, fp);
    if (hipGetLastError() != hipSuccess) ok = false;
  }
  if (ok && hipMemcpyAsync(&failed, fd.fail, 4, hipMemcpyDeviceToHost, s) != hipSuccess) ok = false;
  if (hipStreamSynchronize(s) != hipSuccess) ok = false;
  for (void* p : tmp) (void)hipFree(p);
  if (!ok) {
    (void)hipGetLastError();
    return fail(DMC_ERR_DEVICE, "device factorisation of the normal matrix failed");
  }
  if (failed != INT32_MAX)
    return fail(DMC_ERR_SINGULAR, "normal matrix is not numerically positive definite (supernode " +
                                      std::to_string(failed - 1) + ")");
  m->dev.chol.brow = fd.B;
  return DMC_OK;
}

dmc_status dmc_mesh_create(dmc_ctx ctx, int32_t n, int32_t n_tris, const int32_t* tris,
                           int32_t n_anchors, const int32_t* anchors, int32_t laplacian,
                           dmc_mesh* out) {
  if (!ctx || !out) return fail(DMC_ERR_INVALID_ARG, "ctx or out is NULL");
  *out = nullptr;
  dmc::HostCsr C, M;
  dmc::CholFactor F;
  double info[DMC_FACTOR_INFO_LEN];
  const auto t_setup = std::chrono::steady_clock::now();
  dmc_status st =
      build_mesh_host(n, n_tris, tris, n_anchors, anchors, laplacian, C, M, F, info, false);
  if (st != DMC_OK) return st;

  std::vector<double> w64(n), dinv(n, 0.0);
  std::vector<float> w32(n);
  std::vector<int32_t> slot(n, -1);
  for (int32_t i = 0; i < n; ++i) {
    const double d = C.rowptr[i + 1] - C.rowptr[i];
    w64[i] = laplacian == DMC_LAP_UNIFORM ? 1.0 / d : d;
    w32[i] = (float)w64[i];
    for (int32_t e = M.rowptr[i]; e < M.rowptr[i + 1]; ++e)
      if (M.col[e] == i) dinv[i] = 1.0 / M.val[e];
  }
  for (int32_t a = 0; a < n_anchors; ++a) slot[anchors[a]] = a;
  // the decoder's row order: the factor's elimination order (position p holds
  // vertex perm[p]); its operators re-indexed by position, each row's entries
  // kept in the vertex's own order (the sums run as in vertex order)
  const std::vector<int32_t>& perm = F.perm;
  std::vector<int32_t> dpos(n), d_rowptr(n + 1, 0), d_col(C.col.size()), d_slot(n),
      d_anchors(n_anchors), pm_rowptr(n + 1, 0), pm_col(M.col.size());
  std::vector<double> d_w64(n), pm_val(M.val.size()), pm_dinv(n);
  for (int32_t q = 0; q < n; ++q) dpos[perm[q]] = q;
  for (int32_t q = 0; q < n; ++q) {
    const int32_t i = perm[q];
    d_w64[q] = w64[i];
    d_slot[q] = slot[i];
    pm_dinv[q] = dinv[i];
    d_rowptr[q + 1] = d_rowptr[q] + (C.rowptr[i + 1] - C.rowptr[i]);
    for (int32_t e = C.rowptr[i], o = d_rowptr[q]; e < C.rowptr[i + 1]; ++e, ++o)
      d_col[o] = dpos[C.col[e]];
    pm_rowptr[q + 1] = pm_rowptr[q] + (M.rowptr[i + 1] - M.rowptr[i]);
    for (int32_t e = M.rowptr[i], o = pm_rowptr[q]; e < M.rowptr[i + 1]; ++e, ++o) {
      pm_col[o] = dpos[M.col[e]];
      pm_val[o] = M.val[e];
    }
  }
  for (int32_t a = 0; a < n_anchors; ++a) d_anchors[a] = dpos[anchors[a]];
  // factor work items: (supernode, first row of a 64-row tile), by level, over
  // the supernode's w columns and over its m rows
  std::vector<int32_t> tw_sn, tw_r0, tm_sn, tm_r0, level_w(F.nlevels + 1, 0),
      level_m(F.nlevels + 1, 0), level_maxw(F.nlevels, 0);
  for (int32_t lv = 0; lv < F.nlevels; ++lv) {
    for (int32_t sn = 0; sn < F.nsuper; ++sn) {
      if (F.sn_level[sn] != lv) continue;
      const int32_t w = F.sn_start[sn + 1] - F.sn_start[sn];
      const int32_t mm = F.sn_rowptr[sn + 1] - F.sn_rowptr[sn];
      level_maxw[lv] = std::max(level_maxw[lv], w);
      for (int32_t r0 = 0; r0 < w; r0 += 64) {
        tw_sn.push_back(sn);
        tw_r0.push_back(r0);
      }
      for (int32_t r0 = 0; r0 < mm; r0 += 64) {
        tm_sn.push_back(sn);
        tm_r0.push_back(r0);
      }
    }
    level_w[lv + 1] = (int32_t)tw_sn.size();
    level_m[lv + 1] = (int32_t)tm_sn.size();
  }

  HIP_TRY(hipSetDevice(ctx->device));
  dmc_mesh m = new dmc_mesh_s();
  m->ctx = ctx;
  bool ok = true;
  auto up = [&](const void* src, size_t bytes) -> void* {
    void* d = nullptr;
    if (hipMalloc(&d, std::max<size_t>(bytes, 8)) != hipSuccess) {
      ok = false;
      return nullptr;
    }
    m->allocations.push_back(d);
    if (bytes && hipMemcpy(d, src, bytes, hipMemcpyHostToDevice) != hipSuccess) ok = false;
    return d;
  };
  dmc::MeshDev& dv = m->dev;
  dv.n = n;
  dv.nnz = (int32_t)C.col.size();
  dv.nc = n_anchors;
  dv.laplacian = laplacian;
  dv.m_nnz = (int32_t)M.col.size();
  dv.rowptr = (const int32_t*)up(C.rowptr.data(), C.rowptr.size() * 4);
  dv.col = (const int32_t*)up(C.col.data(), C.col.size() * 4);
  dv.w64 = (const double*)up(w64.data(), n * 8);
  dv.w32 = (const float*)up(w32.data(), n * 4);
  dv.anchors = (const int32_t*)up(anchors, (size_t)n_anchors * 4);
  dv.dpos = (const int32_t*)up(dpos.data(), n * 4);
  dv.d_rowptr = (const int32_t*)up(d_rowptr.data(), d_rowptr.size() * 4);
  dv.d_col = (const int32_t*)up(d_col.data(), d_col.size() * 4);
  dv.d_w64 = (const double*)up(d_w64.data(), n * 8);
  dv.d_slot = (const int32_t*)up(d_slot.data(), n * 4);
  dv.d_anchors = (const int32_t*)up(d_anchors.data(), (size_t)n_anchors * 4);
  dv.m_rowptr = (const int32_t*)up(pm_rowptr.data(), pm_rowptr.size() * 4);
  pm_col.resize(pm_col.size() + dmc::kMatPad, 0);
  pm_val.resize(pm_val.size() + dmc::kMatPad, 0.0);
  dv.m_col = (const int32_t*)up(pm_col.data(), pm_col.size() * 4);
  dv.m_val = (const double*)up(pm_val.data(), pm_val.size() * 8);
  dv.m_dinv = (const double*)up(pm_dinv.data(), n * 8);
  dmc::CholDev& cd = dv.chol;
  dv.solve_entries = info[6];
  cd.n = n;
  cd.ns = F.nsuper;
  cd.nlevels = F.nlevels;
  cd.nslots = F.slot_base[F.nsuper];
  cd.perm = (const int32_t*)up(F.perm.data(), F.perm.size() * 4);
  cd.sn_start = (const int32_t*)up(F.sn_start.data(), F.sn_start.size() * 4);
  cd.sn_rowptr = (const int32_t*)up(F.sn_rowptr.data(), F.sn_rowptr.size() * 4);
  cd.rowidx = (const int32_t*)up(F.rowidx.data(), F.rowidx.size() * 4);
  cd.sn_valptr = (const int64_t*)up(F.sn_valptr.data(), F.sn_valptr.size() * 8);
  cd.slot_base = (const int64_t*)up(F.slot_base.data(), F.slot_base.size() * 8);
  cd.contrib_ptr = (const int32_t*)up(F.contrib_ptr.data(), F.contrib_ptr.size() * 4);
  cd.contrib_slot = (const int32_t*)up(F.contrib_slot.data(), F.contrib_slot.size() * 4);
  cd.task_w_sn = (const int32_t*)up(tw_sn.data(), tw_sn.size() * 4);
  cd.task_w_r0 = (const int32_t*)up(tw_r0.data(), tw_r0.size() * 4);
  cd.task_m_sn = (const int32_t*)up(tm_sn.data(), tm_sn.size() * 4);
  cd.task_m_r0 = (const int32_t*)up(tm_r0.data(), tm_r0.size() * 4);
  m->level_w = level_w;
  m->level_m = level_m;
  m->level_maxw = level_maxw;
  cd.level_w_host = m->level_w.data();
  cd.level_m_host = m->level_m.data();
  cd.level_maxw_host = m->level_maxw.data();
  if (!ok) {
    for (void* p : m->allocations) (void)hipFree(p);
    delete m;
    (void)hipGetLastError();
    return fail(DMC_ERR_OUT_OF_MEMORY, "cannot upload mesh");
  }
  st = factor_on_device(ctx, m, F);
  if (st != DMC_OK) {
    (void)hipStreamSynchronize(ctx->stream);
    for (void* p : m->allocations) (void)hipFree(p);
    delete m;
    return st;
  }
  info[5] = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_setup).count();
  std::memcpy(m->factor_info, info, sizeof(info));
  st = build_anchor_response(ctx, m);
  if (st != DMC_OK) {
    (void)hipStreamSynchronize(ctx->stream);
    for (void* p : m->allocations) (void)hipFree(p);
    delete m;
    return st;
  }
  ctx->meshes.push_back(m);
  *out = m;
  return DMC_OK;
}

int32_t dmc_mesh_anchor_response(dmc_mesh mesh, int32_t* cg_iters, double* resid) {
  if (!mesh) return 0;
  if (cg_iters) *cg_iters = mesh->g_iters;
  if (resid) *resid = mesh->dev.G_resid;
  return mesh->dev.G ? 1 : 0;
}

void dmc_mesh_factor_info(dmc_mesh mesh, double info[DMC_FACTOR_INFO_LEN]) {
  if (!mesh || !info) return;
  std::memcpy(info, mesh->factor_info, sizeof(mesh->factor_info));
}

dmc_status dmc_host_normal_solve(int32_t n, int32_t n_tris, const int32_t* tris, int32_t n_anchors,
                                 const int32_t* anchors, int32_t laplacian, int32_t ncols,
                                 const double* B, double* X, double info[DMC_FACTOR_INFO_LEN]) {
  if (ncols < 1 || !B || !X) return fail(DMC_ERR_INVALID_ARG, "bad right-hand side");
  dmc::HostCsr C, M;
  dmc::CholFactor F;
  double inf[DMC_FACTOR_INFO_LEN];
  dmc_status st =
      build_mesh_host(n, n_tris, tris, n_anchors, anchors, laplacian, C, M, F, inf, true);
  if (st != DMC_OK) return st;
  dmc::chol_solve_host(F, ncols, B, X);
  if (info) std::memcpy(info, inf, sizeof(inf));
  return DMC_OK;
}

void dmc_mesh_destroy(dmc_mesh mesh) {
  if (!mesh) return;
  dmc_ctx ctx = mesh->ctx;
  (void)hipStreamSynchronize(ctx->stream);
  for (void* p : mesh->allocations) (void)hipFree(p);
  ctx->meshes.erase(std::remove(ctx->meshes.begin(), ctx->meshes.end(), mesh), ctx->meshes.end());
  delete mesh;
}

int32_t dmc_mesh_nnz(dmc_mesh mesh) { return mesh ? mesh->dev.nnz : 0; }
int32_t dmc_mesh_normal_nnz(dmc_mesh mesh) { return mesh ? mesh->dev.m_nnz : 0; }

size_t dmc_window_code_bytes(int32_t n, int32_t T, int32_t n_anchors, const dmc_params* p) {
  if (!p || n < 1 || T < 1 || n_anchors < 0) return 0;
  return dmc::record_layout(n, T, std::min(p->k, T), n_anchors, *p).bytes;
}

size_t dmc_sequence_code_bytes(int32_t n, int32_t F, int32_t T, int32_t n_anchors,
                               const dmc_params* p) {
  if (!p || F < 1 || T < 1) return 0;
  const int32_t nw = F / T, tail = F % T;
  size_t b = (size_t)nw * dmc_window_code_bytes(n, T, n_anchors, p);
  if (tail) b += dmc_window_code_bytes(n, tail, n_anchors, p);
  return b;
}

}  // extern "C"

namespace {

// Scratch of one window's encode: the chain's pieces (autocorrelation
// partials, R, dictionary, coefficients), and the window's stats when the
// caller's array holds them too (o_stats).
struct WindowScratch {
  size_t o_chain = 0, o_stats = 0, total = 0;
};

WindowScratch window_scratch(const dmc::MeshDev& m, int32_t T, const dmc_params& p,
                             bool with_stats) {
  Carve cv;
  WindowScratch w;
  w.o_chain = cv.add(chain_scratch_bytes(m.n, T, 1, std::min(p.k, T), p.precision, p.init));
  if (with_stats) w.o_stats = cv.add(sizeof(dmc::StatsDev));
  w.total = cv.total();
  return w;
}

// dmc_encode_window on a given scratch area and stats slot (checked
// arguments; ws holds window_scratch(...).total bytes).
dmc_status encode_window_on(dmc_ctx ctx, const dmc::MeshDev& m, const void* frames, int32_t T,
                            const dmc_params& p, const void* q_start, void* code, void* u_out,
                            void* coef_out, dmc_window_stats* stats, uint8_t* ws,
                            const WindowScratch& wl, dmc::StatsDev* sd) {
  const dmc::RecordLayout lay = dmc::record_layout(m.n, T, p.k, m.nc, p);
  if (stats) HIP_TRY(hipEventRecord(ctx->ev[0], ctx->stream));
  dmc_status st = encode_chain(ctx, m, frames, T, 1, p.k, p, q_start, (uint8_t*)code, lay, u_out,
                               coef_out, ws + wl.o_chain, sd);
  if (st != DMC_OK) return st;
  if (stats) HIP_TRY(hipEventRecord(ctx->ev[1], ctx->stream));
  // the convergence of the orthogonal iterations is read back at this one
  // synchronisation point, whether or not stats are requested
  HIP_TRY(hipMemcpyAsync(ctx->pinned, sd, sizeof(dmc::StatsDev), hipMemcpyDeviceToHost,
                         ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  const dmc::StatsDev hs = *(const dmc::StatsDev*)ctx->pinned;
  if (stats) {
    std::vector<std::vector<uint8_t>> heads;
    st = read_record_heads(ctx, (const uint8_t*)code, 1, lay, nullptr, heads);
    if (st != DMC_OK) return st;
    std::memset(stats, 0, sizeof(*stats));
    fill_stats(stats, hs, lay, heads[0].data());
    stats->ms_encode = elapsed_ms(ctx->ev[0], ctx->ev[1]);
  }
  if (oi_not_converged(&hs, 1, p.oi_tol))
    return fail(DMC_ERR_NOT_CONVERGED, "orthogonal iterations ended above oi_tol");
  return DMC_OK;
}

dmc_status check_encode_window(dmc_ctx ctx, dmc_mesh mesh, const void* frames, int32_t T,
                               const dmc_params* params, void* code) {
  if (!ctx || !mesh || !frames || !code) return fail(DMC_ERR_INVALID_ARG, "NULL argument");
  dmc_status st = check_params(params, T);
  if (st != DMC_OK) return st;
  if (params->k > T) return fail(DMC_ERR_INVALID_ARG, "k must not exceed T");
  return check_learned(ctx, *params, T);
}

}  // namespace

extern "C" {

dmc_status dmc_encode_window(dmc_ctx ctx, dmc_mesh mesh, const void* frames, int32_t T,
                             const dmc_params* params, const void* q_start, void* code,
                             void* u_out, void* coef_out, dmc_window_stats* stats) {
  dmc_status st = check_encode_window(ctx, mesh, frames, T, params, code);
  if (st != DMC_OK) return st;
  HIP_TRY(hipSetDevice(ctx->device));
  const WindowScratch wl = window_scratch(mesh->dev, T, *params, false);
  st = ensure_scratch(ctx, wl.total);
  if (st != DMC_OK) return st;
  st = ensure_stats(ctx, sizeof(dmc::StatsDev));
  if (st != DMC_OK) return st;
  return encode_window_on(ctx, mesh->dev, frames, T, *params, q_start, code, u_out, coef_out,
                          stats, (uint8_t*)ctx->scratch, wl, (dmc::StatsDev*)ctx->stats);
}

dmc_status dmc_encode_window_noalloc(dmc_ctx ctx, dmc_mesh mesh, const void* frames, int32_t T,
                                     const dmc_params* params, const void* q_start, void* code,
                                     void* u_out, void* coef_out, dmc_window_stats* stats) {
  dmc_status st = check_encode_window(ctx, mesh, frames, T, params, code);
  if (st != DMC_OK) return st;
  const WindowScratch wl = window_scratch(mesh->dev, T, *params, true);
  if (wl.total > kNoAllocScratchBytes)
    return fail(DMC_ERR_BUFFER_TOO_SMALL,
                "this window needs " + std::to_string(wl.total) +
                    " bytes of scratch; the fixed array of dmc_encode_window_noalloc holds " +
                    std::to_string(kNoAllocScratchBytes));
  HIP_TRY(hipSetDevice(ctx->device));
  uint8_t* ws = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    ws = (uint8_t*)g_noalloc_scratch[ctx->device];
  }
  if (!ws) return fail(DMC_ERR_DEVICE, "no address of the fixed scratch for this device");
  return encode_window_on(ctx, mesh->dev, frames, T, *params, q_start, code, u_out, coef_out,
                          stats, ws, wl, (dmc::StatsDev*)(ws + wl.o_stats));
}

static dmc::SeqLayout seq_layout(int32_t n, int32_t F, int32_t T, int32_t nc, const dmc_params& p) {
  dmc::SeqLayout sl;
  sl.T = T;
  sl.nw_full = F / T;
  sl.T_tail = F % T;
  sl.full = dmc::record_layout(n, T, std::min(p.k, T), nc, p);
  sl.tail = dmc::record_layout(n, std::max(sl.T_tail, 1), std::min(p.k, std::max(sl.T_tail, 1)),
                               nc, p);
  sl.rec_bytes_full = sl.full.bytes;
  return sl;
}

// The decoder indexes a record by the sizes and formats of the call, so every
// window's header (written by k_header) is read back and compared with them
// before any decode kernel runs.
dmc_status check_headers(dmc_ctx ctx, const dmc::MeshDev& m, const uint8_t* records,
                         const dmc::SeqLayout& sl, bool standalone = false) {
  const int32_t nw = sl.nw_full + (sl.T_tail ? 1 : 0);
  dmc_status st = ensure_pinned(ctx, (size_t)nw * 64);
  if (st != DMC_OK) return st;
  uint8_t* h = (uint8_t*)ctx->pinned;
  if (sl.nw_full)
    HIP_TRY(hipMemcpy2DAsync(h, 64, records, sl.rec_bytes_full, 64, sl.nw_full,
                             hipMemcpyDeviceToHost, ctx->stream));
  if (sl.T_tail)
    HIP_TRY(hipMemcpyAsync(h + (size_t)sl.nw_full * 64,
                           records + (size_t)sl.nw_full * sl.rec_bytes_full, 64,
                           hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  for (int32_t w = 0; w < nw; ++w) {
    const dmc::RecordLayout& l = w < sl.nw_full ? sl.full : sl.tail;
    int32_t hd[16];
    std::memcpy(hd, h + (size_t)w * 64, sizeof(hd));
    const int32_t want[10] = {dmc::kRecordMagic, l.T,          l.k,         m.n,         m.nc,
                              l.coef_bits,       l.anchor_bits, l.dict_bits, l.precision, l.dict_mode};
    static const char* what[10] = {"magic",       "T",         "k",         "n",
                                   "n_c",         "coef_bits", "anchor_bits", "dict_bits",
                                   "precision",   "dict_mode"};
    for (int f = 0; f < 10; ++f)
      if (hd[f] != want[f])
        return fail(DMC_ERR_INVALID_ARG, "record of window " + std::to_string(w) + ": header " +
                                             what[f] + " = " + std::to_string(hd[f]) +
                                             ", the call expects " + std::to_string(want[f]));
    uint64_t step_bits;
    std::memcpy(&step_bits, &hd[dmc::kHdrStepLo], 8);
    double step;
    std::memcpy(&step, &step_bits, 8);
    if (step != l.coef_step)
      return fail(DMC_ERR_INVALID_ARG, "record of window " + std::to_string(w) +
                                           ": coef_step differs from the call's");
    if (standalone && hd[dmc::kHdrHasDiff])
      return fail(DMC_ERR_INVALID_ARG, "the record codes its dictionary as differences from "
                                       "the previous window's: decode it with its sequence");
  }
  return DMC_OK;
}

dmc_status dmc_decode_window(dmc_ctx ctx, dmc_mesh mesh, const void* code, int32_t T,
                             const dmc_params* params, void* frames_out, dmc_window_stats* stats) {
  if (!ctx || !mesh || !code || !frames_out) return fail(DMC_ERR_INVALID_ARG, "NULL argument");
  dmc_status st = check_params(params, T, true);
  if (st != DMC_OK) return st;
  HIP_TRY(hipSetDevice(ctx->device));
  const dmc::SeqLayout sl = seq_layout(mesh->dev.n, T, T, mesh->dev.nc, *params);
  st = check_headers(ctx, mesh->dev, (const uint8_t*)code, sl, true);
  if (st != DMC_OK) return st;
  int32_t iters = 0;
  double res = 0.0;
  if (stats) HIP_TRY(hipEventRecord(ctx->ev[1], ctx->stream));
  st = decode_all(ctx, mesh->dev, (const uint8_t*)code, sl, *params, frames_out, &iters, &res);
  if (st != DMC_OK && st != DMC_ERR_NOT_CONVERGED) return st;
  if (stats) {
    HIP_TRY(hipEventRecord(ctx->ev[2], ctx->stream));
    HIP_TRY(hipEventSynchronize(ctx->ev[2]));
    std::vector<std::vector<uint8_t>> heads;
    dmc_status hst = read_record_heads(ctx, (const uint8_t*)code, 1, sl.full, nullptr, heads);
    if (hst != DMC_OK) return hst;
    std::memset(stats, 0, sizeof(*stats));
    stats->T = T;
    stats->k = std::min(params->k, T);
    fill_bits(stats, sl.full, heads[0].data());
    stats->cg_iters = iters;
    stats->cg_resid = res;
    stats->ms_decode = elapsed_ms(ctx->ev[1], ctx->ev[2]);
  }
  return st;
}

dmc_status dmc_decode_sequence(dmc_ctx ctx, dmc_mesh mesh, const void* codes, int32_t F,
                               int32_t T, const dmc_params* params, void* frames_out,
                               dmc_window_stats* per_window) {
  if (!ctx || !mesh || !codes || !frames_out) return fail(DMC_ERR_INVALID_ARG, "NULL argument");
  if (F < 1) return fail(DMC_ERR_INVALID_ARG, "F must be >= 1");
  dmc_status st = check_params(params, T, true);
  if (st != DMC_OK) return st;
  HIP_TRY(hipSetDevice(ctx->device));
  const dmc::SeqLayout sl = seq_layout(mesh->dev.n, F, T, mesh->dev.nc, *params);
  st = check_headers(ctx, mesh->dev, (const uint8_t*)codes, sl);
  if (st != DMC_OK) return st;
  int32_t iters = 0;
  double res = 0.0;
  if (per_window) HIP_TRY(hipEventRecord(ctx->ev[1], ctx->stream));
  st = decode_all(ctx, mesh->dev, (const uint8_t*)codes, sl, *params, frames_out, &iters, &res);
  if (st != DMC_OK && st != DMC_ERR_NOT_CONVERGED) return st;
  if (per_window) {
    HIP_TRY(hipEventRecord(ctx->ev[2], ctx->stream));
    HIP_TRY(hipEventSynchronize(ctx->ev[2]));
    const float ms = elapsed_ms(ctx->ev[1], ctx->ev[2]);
    const int nw = sl.nw_full + (sl.T_tail ? 1 : 0);
    std::vector<std::vector<uint8_t>> heads;
    dmc_status hst = read_record_heads(ctx, (const uint8_t*)codes, sl.nw_full, sl.full,
                                       sl.T_tail ? &sl.tail : nullptr, heads);
    if (hst != DMC_OK) return hst;
    for (int w = 0; w < nw; ++w) {
      const dmc::RecordLayout& l = w < sl.nw_full ? sl.full : sl.tail;
      std::memset(&per_window[w], 0, sizeof(dmc_window_stats));
      per_window[w].T = l.T;
      per_window[w].k = l.k;
      fill_bits(&per_window[w], l, heads[w].data());
      per_window[w].cg_iters = iters;
      per_window[w].cg_resid = res;
      per_window[w].ms_decode = ms;
    }
  }
  return st;
}

// Scratch bytes of the encoder (the chains of full windows and of the short
// last window) and of the decoder (the solve's vectors), for an F-frame
// sequence; the two never live together.
size_t encode_scratch_bytes(const dmc::MeshDev& m, const dmc::SeqLayout& sl, const dmc_params& p,
                            size_t* o_full = nullptr, size_t* o_tail = nullptr) {
  const int32_t F = sl.nw_full * sl.T + sl.T_tail;
  Carve cv;
  (void)F;
  const size_t of = cv.add(sl.nw_full ? chain_scratch_bytes(m.n, sl.T, sl.nw_full, sl.full.k,
                                                              p.precision, p.init)
                                      : 0);
  const size_t ot = cv.add(sl.T_tail ? chain_scratch_bytes(m.n, sl.T_tail, 1, sl.tail.k,
                                                             p.precision, DMC_INIT_EXACT)
                                     : 0);
  if (o_full) *o_full = of;
  if (o_tail) *o_tail = ot;
  return cv.total();
}

dmc_status dmc_compress_sequence(dmc_ctx ctx, dmc_mesh mesh, const void* frames, int32_t F,
                                 int32_t T, const dmc_params* params, const void* q_start,
                                 void* codes, size_t codes_bytes, void* frames_out,
                                 dmc_window_stats* per_window) {
  if (!ctx || !mesh || !frames || !codes) return fail(DMC_ERR_INVALID_ARG, "NULL argument");
  if (F < 1) return fail(DMC_ERR_INVALID_ARG, "F must be >= 1");
  dmc_status st = check_params(params, T);
  if (st != DMC_OK) return st;
  const dmc_params& p = *params;
  if ((p.init == DMC_INIT_RANDOM || p.init == DMC_INIT_SKETCH) && !q_start && F >= T)
    return fail(DMC_ERR_INVALID_ARG, "DMC_INIT_RANDOM and DMC_INIT_SKETCH need q_start");
  const dmc::MeshDev& m = mesh->dev;
  const dmc::SeqLayout sl = seq_layout(m.n, F, T, m.nc, p);
  const size_t need = dmc_sequence_code_bytes(m.n, F, T, m.nc, &p);
  if (codes_bytes < need)
    return fail(DMC_ERR_BUFFER_TOO_SMALL, "codes buffer needs " + std::to_string(need) + " bytes");
  HIP_TRY(hipSetDevice(ctx->device));
  const int32_t nw = sl.nw_full + (sl.T_tail ? 1 : 0);
  const int32_t k_full = std::min(p.k, T);
  if (sl.nw_full) {
    st = check_learned(ctx, p, T);
    if (st != DMC_OK) return st;
  }
  dmc_params p_tail = p;  // a shorter last window starts from its exact eigenvectors
  p_tail.init = DMC_INIT_EXACT;
  size_t o_full = 0, o_tail = 0;
  st = ensure_scratch(ctx, encode_scratch_bytes(m, sl, p, &o_full, &o_tail));
  if (st != DMC_OK) return st;
  st = ensure_stats(ctx, sizeof(dmc::StatsDev) * nw);
  if (st != DMC_OK) return st;
  // the stats are staged in the upper half of the staging buffer, apart from
  // the decoder's convergence flags in the lower half
  const size_t stats_at =
      frames_out ? std::max(kPinnedBytes / 2,
                            dmc::align_up((size_t)decode_plan(m, sl, p).ncols * 12 + 4096))
                 : 0;
  st = ensure_pinned(ctx, stats_at + sizeof(dmc::StatsDev) * nw);
  if (st != DMC_OK) return st;
  uint8_t* ws = (uint8_t*)ctx->scratch;
  dmc::StatsDev* sd = (dmc::StatsDev*)ctx->stats;
  if (per_window) HIP_TRY(hipEventRecord(ctx->ev[0], ctx->stream));
  const size_t rs = real_size(p.precision);
  if (sl.nw_full) {
    st = encode_chain(ctx, m, frames, T, sl.nw_full, k_full, p, q_start, (uint8_t*)codes, sl.full,
                      nullptr, nullptr, ws + o_full, sd);
    if (st != DMC_OK) return st;
  }
  if (sl.T_tail) {
    const size_t f0 = (size_t)sl.nw_full * T;
    st = encode_chain(ctx, m, (const uint8_t*)frames + f0 * 3 * m.n * rs, sl.T_tail, 1, sl.tail.k,
                      p_tail, nullptr, (uint8_t*)codes + (size_t)sl.nw_full * sl.full.bytes, sl.tail,
                      nullptr, nullptr, ws + o_tail,
                      sd + sl.nw_full);
    if (st != DMC_OK) return st;
  }
  if (per_window) HIP_TRY(hipEventRecord(ctx->ev[1], ctx->stream));
  // the windows' convergence is staged now and read at the one
  // synchronisation point at the end
  uint8_t* staged = (uint8_t*)ctx->pinned + stats_at;
  HIP_TRY(hipMemcpyAsync(staged, sd, sizeof(dmc::StatsDev) * nw, hipMemcpyDeviceToHost,
                         ctx->stream));
  int32_t iters = 0;
  double res = 0.0;
  dmc_status dst = DMC_OK;
  if (frames_out) {
    dst = decode_all(ctx, m, (const uint8_t*)codes, sl, p, frames_out, &iters, &res);
    if (dst != DMC_OK && dst != DMC_ERR_NOT_CONVERGED) return dst;
  }
  if (per_window) HIP_TRY(hipEventRecord(ctx->ev[2], ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  std::vector<dmc::StatsDev> hs(nw);
  std::memcpy(hs.data(), staged, sizeof(dmc::StatsDev) * nw);
  if (per_window) {
    const float ms_enc = elapsed_ms(ctx->ev[0], ctx->ev[1]);
    const float ms_dec = frames_out ? elapsed_ms(ctx->ev[1], ctx->ev[2]) : 0.f;
    std::vector<std::vector<uint8_t>> heads;
    st = read_record_heads(ctx, (const uint8_t*)codes, sl.nw_full, sl.full,
                           sl.T_tail ? &sl.tail : nullptr, heads);
    if (st != DMC_OK) return st;
    for (int w = 0; w < nw; ++w) {
      std::memset(&per_window[w], 0, sizeof(dmc_window_stats));
      const bool tail = w >= sl.nw_full;
      fill_stats(&per_window[w], hs[w], tail ? sl.tail : sl.full, heads[w].data());
      per_window[w].cg_iters = iters;
      per_window[w].cg_resid = res;
      per_window[w].ms_encode = ms_enc;
      per_window[w].ms_decode = ms_dec;
    }
  }
  if (dst != DMC_OK) return dst;
  if (oi_not_converged(hs.data(), nw, p.oi_tol))
    return fail(DMC_ERR_NOT_CONVERGED, "orthogonal iterations ended above oi_tol");
  return DMC_OK;
}

size_t dmc_workspace_bytes(dmc_mesh mesh, int32_t F, int32_t T, const dmc_params* params) {
  if (!mesh || !params || F < 1 || T < 1 || T > 64 || params->k < 1) return 0;
  const dmc::MeshDev& m = mesh->dev;
  const dmc::SeqLayout sl = seq_layout(m.n, F, T, m.nc, *params);
  const size_t enc = encode_scratch_bytes(m, sl, *params);
  const size_t dec = decode_plan(m, sl, *params).lay.total;
  return std::max(enc, dec);
}

dmc_status dmc_delta(dmc_ctx ctx, dmc_mesh mesh, const void* frames, int32_t F, int32_t precision,
                     void* out) {
  if (!ctx || !mesh || !frames || !out) return fail(DMC_ERR_INVALID_ARG, "NULL argument");
  if (F < 1) return fail(DMC_ERR_INVALID_ARG, "F must be >= 1");
  if (precision != DMC_FP64 && precision != DMC_FP32 && precision != DMC_BF16)
    return fail(DMC_ERR_INVALID_ARG, "bad precision");
  HIP_TRY(hipSetDevice(ctx->device));
  dmc::launch_delta(ctx->stream, mesh->dev, frames, out, F, precision);
  return check_launch("delta");
}

dmc_status dmc_autocorrelation(dmc_ctx ctx, dmc_mesh mesh, const void* frames, int32_t T,
                               int32_t precision, void* R_out) {
  if (!ctx || !mesh || !frames || !R_out) return fail(DMC_ERR_INVALID_ARG, "NULL argument");
  if (T < 1 || T > 64) return fail(DMC_ERR_INVALID_ARG, "T must be in 1..64");
  if (precision != DMC_FP64 && precision != DMC_FP32 && precision != DMC_BF16)
    return fail(DMC_ERR_INVALID_ARG, "bad precision");
  HIP_TRY(hipSetDevice(ctx->device));
  dmc_status st = ensure_scratch(ctx, dmc::autocorr_scratch_bytes(mesh->dev.n, T, 1, precision));
  if (st != DMC_OK) return st;
  dmc::launch_autocorr(ctx->stream, frames, mesh->dev.n, T, 1, precision, ctx->scratch,
                       (double*)R_out);
  return check_launch("autocorrelation");
}

dmc_status dmc_mesh_normal_solve(dmc_ctx ctx, dmc_mesh mesh, int32_t ncols, const double* B,
                                 double* X) {
  if (!ctx || !mesh || !B || !X) return fail(DMC_ERR_INVALID_ARG, "NULL argument");
  if (ncols < 1) return fail(DMC_ERR_INVALID_ARG, "ncols must be >= 1");
  if (B == X) return fail(DMC_ERR_INVALID_ARG, "B and X may not alias");
  HIP_TRY(hipSetDevice(ctx->device));
  const dmc::MeshDev& m = mesh->dev;
  const size_t vec = (size_t)m.n * ncols * 8;
  Carve cv;
  const size_t o_b = cv.add(vec), o_z = cv.add(vec), o_w = cv.add(vec), o_y = cv.add(vec);
  const size_t o_u = cv.add((size_t)m.chol.nslots * ncols * 8);
  const size_t o_s = cv.add(dmc::chol_split_bytes(m.chol, ncols));
  dmc_status st = ensure_scratch(ctx, cv.total());
  if (st != DMC_OK) return st;
  uint8_t* ws = (uint8_t*)ctx->scratch;
  hipStream_t s = ctx->stream;
  double* bp = (double*)(ws + o_b);
  double* zp = (double*)(ws + o_z);
  const size_t split = dmc::chol_split_bytes(m.chol, ncols);
  // rows into the factor's order, the two supernodal solves, rows back
  dmc::launch_permute_rows(s, B, m.chol.perm, m.n, ncols, bp);
  dmc::launch_chol_solve(s, m.chol, ncols, bp, zp, (double*)(ws + o_w), (double*)(ws + o_y),
                         (double*)(ws + o_u), split ? (double*)(ws + o_s) : nullptr);
  dmc::launch_permute_rows(s, zp, m.dpos, m.n, ncols, X);
  st = check_launch("normal solve");
  if (st != DMC_OK) return st;
  HIP_TRY(hipStreamSynchronize(s));
  return DMC_OK;
}

}  // extern "C"

// ---- learned start ---------------------------------------------------------

int32_t dmc_mlp_param_count(int32_t k) { return (k < 1 || k > 32) ? 0 : dmc::mlp_param_count(k); }

dmc_status dmc_learned_start(dmc_ctx ctx, int32_t T, int32_t k, const double* omega,
                             const float* theta) {
  if (!ctx) return fail(DMC_ERR_INVALID_ARG, "NULL context");
  if (!omega || !theta) {
    ctx->learned_omega = nullptr;
    ctx->learned_theta = nullptr;
    ctx->learned_T = ctx->learned_k = 0;
    return DMC_OK;
  }
  if (T < 1 || T > 64 || k < 1 || k > 32 || k > T)
    return fail(DMC_ERR_INVALID_ARG, "need 1 <= k <= min(T, 32) and T <= 64");
  ctx->learned_T = T;
  ctx->learned_k = k;
  ctx->learned_omega = omega;
  ctx->learned_theta = theta;
  return DMC_OK;
}

dmc_status dmc_mlp_sketch(dmc_ctx ctx, const double* R, int32_t nb, int32_t T, const double* omega,
                          float* S) {
  if (!ctx || !R || !omega || !S) return fail(DMC_ERR_INVALID_ARG, "NULL argument");
  if (nb < 0 || T < 1 || T > 64) return fail(DMC_ERR_INVALID_ARG, "need nb >= 0 and T in 1..64");
  if (nb == 0) return DMC_OK;
  HIP_TRY(hipSetDevice(ctx->device));
  dmc::launch_mlp_sketch(ctx->stream, R, nb, T, omega, S);
  return check_launch("mlp sketch");
}

dmc_status dmc_mlp_forward(dmc_ctx ctx, const float* theta, int32_t k, const float* S, int32_t N,
                           float* Q, float* cache) {
  if (!ctx || !theta || !S || !Q) return fail(DMC_ERR_INVALID_ARG, "NULL argument");
  if (k < 1 || k > 32 || N < 0) return fail(DMC_ERR_INVALID_ARG, "need k in 1..32 and N >= 0");
  if (N == 0) return DMC_OK;
  HIP_TRY(hipSetDevice(ctx->device));
  dmc::launch_mlp_forward(ctx->stream, theta, k, S, N, Q, cache);
  return check_launch("mlp forward");
}

dmc_status dmc_mlp_loss_grad(dmc_ctx ctx, const float* Q, const double* U, int32_t nb, int32_t T,
                             int32_t k, double mu, float* dQ, double* loss) {
  if (!ctx || !Q || !U || !dQ) return fail(DMC_ERR_INVALID_ARG, "NULL argument");
  if (nb < 1 || T < 1 || T > 64 || k < 1 || k > 32 || k > T)
    return fail(DMC_ERR_INVALID_ARG, "need nb >= 1, T in 1..64, 1 <= k <= min(T, 32)");
  if (!(mu >= 0.0)) return fail(DMC_ERR_INVALID_ARG, "mu must be >= 0");
  HIP_TRY(hipSetDevice(ctx->device));
  dmc::launch_mlp_loss(ctx->stream, Q, U, T, k, nb, mu, dQ, loss);
  return check_launch("mlp loss");
}

dmc_status dmc_mlp_backward(dmc_ctx ctx, const float* theta, int32_t k, const float* S, int32_t N,
                            const float* cache, const float* dQ, float* grad) {
  if (!ctx || !theta || !S || !cache || !dQ || !grad)
    return fail(DMC_ERR_INVALID_ARG, "NULL argument");
  if (k < 1 || k > 32 || N < 1) return fail(DMC_ERR_INVALID_ARG, "need k in 1..32 and N >= 1");
  HIP_TRY(hipSetDevice(ctx->device));
  Carve cv;
  const size_t o_part = cv.add((size_t)dmc::mlp_bwd_parts() * dmc::mlp_param_count(k) * sizeof(float));
  const size_t o_dz = cv.add((size_t)N * 256 * sizeof(float));
  dmc_status st = ensure_scratch(ctx, cv.total());
  if (st != DMC_OK) return st;
  uint8_t* ws = (uint8_t*)ctx->scratch;
  dmc::launch_mlp_backward(ctx->stream, theta, k, S, N, cache, dQ, (float*)(ws + o_dz),
                           (float*)(ws + o_part), grad);
  return check_launch("mlp backward");
}

dmc_status dmc_mlp_adam(dmc_ctx ctx, float* theta, const float* grad, float* m, float* v,
                        int32_t count, int32_t step, double lr, double beta1, double beta2,
                        double eps) {
  if (!ctx || !theta || !grad || !m || !v) return fail(DMC_ERR_INVALID_ARG, "NULL argument");
  if (count < 1 || step < 1 || !(lr > 0.0) || !(beta1 >= 0.0 && beta1 < 1.0) ||
      !(beta2 >= 0.0 && beta2 < 1.0) || !(eps >= 0.0))
    return fail(DMC_ERR_INVALID_ARG, "bad Adam arguments");
  HIP_TRY(hipSetDevice(ctx->device));
  dmc::launch_mlp_adam(ctx->stream, theta, grad, m, v, count, step, lr, beta1, beta2, eps);
  return check_launch("mlp adam");
}

// ---- orthogonal iterations on independent covariance blocks ----------------

dmc_status dmc_oi_blocks(dmc_ctx ctx, const double* R, int32_t nb, int32_t T,
                         const dmc_params* params, const void* q_start, double* U_out,
                         int32_t* sweeps, double* resid) {
  if (!ctx || !R || !U_out) return fail(DMC_ERR_INVALID_ARG, "NULL argument");
  if (nb < 1) return fail(DMC_ERR_INVALID_ARG, "nb must be >= 1");
  dmc_status st = check_params(params, T);
  if (st != DMC_OK) return st;
  const dmc_params& p = *params;
  if (p.k > T) return fail(DMC_ERR_INVALID_ARG, "k must not exceed T");
  if (p.init == DMC_INIT_PREV)
    return fail(DMC_ERR_INVALID_ARG, "independent blocks take DMC_INIT_RANDOM, _SKETCH, _EXACT "
                                     "or _LEARNED");
  if ((p.init == DMC_INIT_RANDOM || p.init == DMC_INIT_SKETCH) && !q_start)
    return fail(DMC_ERR_INVALID_ARG, "DMC_INIT_RANDOM and DMC_INIT_SKETCH need q_start");
  st = check_learned(ctx, p, T);
  if (st != DMC_OK) return st;
  HIP_TRY(hipSetDevice(ctx->device));
  Carve cv;
  const bool learned = p.init == DMC_INIT_LEARNED;
  const size_t o_s = cv.add(learned ? (size_t)nb * T * 32 * 4 : 0);
  const size_t o_q = cv.add(learned ? (size_t)nb * T * p.k * 4 : 0);
  st = ensure_scratch(ctx, cv.total());
  if (st != DMC_OK) return st;
  st = ensure_stats(ctx, sizeof(dmc::StatsDev) * nb);
  if (st != DMC_OK) return st;
  uint8_t* ws = (uint8_t*)ctx->scratch;
  if (learned) {
    dmc::launch_mlp_sketch(ctx->stream, R, nb, T, ctx->learned_omega, (float*)(ws + o_s));
    dmc::launch_mlp_forward(ctx->stream, ctx->learned_theta, p.k, (const float*)(ws + o_s), nb * T,
                            (float*)(ws + o_q), nullptr);
  }
  dmc::OiArgs oa{};
  oa.R = R;
  oa.nw = nb;
  oa.T = T;
  oa.k = p.k;
  oa.precision = DMC_FP64;  // blocks and outputs are float64
  oa.init = p.init;
  oa.ncoord = 1;
  oa.q_start = p.init == DMC_INIT_EXACT ? nullptr : q_start;
  oa.q_learned = learned ? (const float*)(ws + o_q) : nullptr;
  oa.u_out = U_out;
  oa.u_canon = nullptr;
  oa.max_sweeps = p.oi_max_sweeps;
  oa.tol = p.oi_tol;
  oa.stats = (dmc::StatsDev*)ctx->stats;
  dmc::launch_oi(ctx->stream, oa);
  st = check_launch("oi blocks");
  if (st != DMC_OK) return st;
  if (sweeps || resid) {
    st = ensure_pinned(ctx, sizeof(dmc::StatsDev) * nb);
    if (st != DMC_OK) return st;
    HIP_TRY(hipMemcpyAsync(ctx->pinned, ctx->stats, sizeof(dmc::StatsDev) * nb,
                           hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    const dmc::StatsDev* hs = (const dmc::StatsDev*)ctx->pinned;
    for (int32_t b = 0; b < nb; ++b) {
      if (sweeps) sweeps[b] = hs[b].sweeps[0];
      if (resid) resid[b] = hs[b].resid[0];
    }
  }
  return DMC_OK;
}

// ---- batched form -----------------------------------------------------------

struct BatchSeq {
  dmc_mesh mesh = nullptr;
  const uint8_t* frames = nullptr;
  int32_t F = 0, T = 0, k_full = 0, k_tail = 0;
  dmc_params p{};
  const void* q_start = nullptr;
  uint8_t* codes = nullptr;
  void* out = nullptr;
  dmc::SeqLayout sl{};
  size_t o_R = 0, o_Rt = 0, o_ut = 0, o_utt = 0;  // covariances, canonical U (full, tail)
  size_t o_ud = 0, o_udt = 0, o_ap = 0, o_apt = 0;  // dequantised dictionaries, anchor partials
  int32_t stats_off = 0;  // first window in the batch's stats array
  int P = 0;              // tuned launch shape
  int branch = 0;         // graph branch the sequence's kernels run on
  int cls[2] = {-1, -1};  // orthogonal-iteration classes of its full windows and tail
};

struct dmc_batch_s {
  dmc_ctx ctx = nullptr;
  int32_t precision = DMC_FP32;
  std::vector<BatchSeq> seq;
  uint8_t* buf = nullptr;
  size_t o_args = 0, o_jobs = 0, o_summary = 0, o_stats = 0;
  std::vector<size_t> o_shared;  // per branch: covariance, projection and decoder scratch
  std::vector<int> cls_tmax, cls_kr, cls_off, cls_n;  // OI launch classes
  hipStream_t stream = nullptr;  // private stream the graph is captured on and replayed on
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  // capture only: one stream per branch, fork and join events of the two
  // per-sequence phases (before and after the orthogonal iterations); one
  // stream and end event per orthogonal-iteration class
  std::vector<hipStream_t> br, cs;
  std::vector<hipEvent_t> ev_fork, ev_join, ev_cls;
  std::vector<int> order2;  // sequences in the order of the second phase
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

// Branch streams wait for what stream s has recorded so far (phase ph).
hipError_t batch_fork(dmc_batch b, hipStream_t s, int ph) {
  if (b->br.empty()) return hipSuccess;
  hipError_t e = hipEventRecord(b->ev_fork[ph], s);
  for (size_t j = 0; j < b->br.size() && e == hipSuccess; ++j)
    e = hipStreamWaitEvent(b->br[j], b->ev_fork[ph], 0);
  return e;
}

// Stream s waits for every branch's work of phase ph.
hipError_t batch_join(dmc_batch b, hipStream_t s, int ph) {
  hipError_t e = hipSuccess;
  const size_t nb = b->br.size();
  for (size_t j = 0; j < nb && e == hipSuccess; ++j) {
    e = hipEventRecord(b->ev_join[ph * nb + j], b->br[j]);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, b->ev_join[ph * nb + j], 0);
  }
  return e;
}

// The whole batch on stream s, with no host synchronisation.  The kernels of
// one sequence run in order on its branch; the branches share nothing but
// the orthogonal-iteration launches between the two phases.
hipError_t batch_enqueue(dmc_batch b, hipStream_t s) {
  const size_t rs = real_size(b->precision);
  auto on = [&](const BatchSeq& q) { return b->br.empty() ? s : b->br[q.branch]; };
  auto shared_of = [&](const BatchSeq& q) { return b->buf + b->o_shared[q.branch]; };
  hipError_t e = batch_fork(b, s, 0);
  if (e != hipSuccess) return e;
  for (BatchSeq& q : b->seq) {
    const dmc::MeshDev& m = q.mesh->dev;
    hipStream_t sq = on(q);
    uint8_t* shared = shared_of(q);
    dmc::launch_write_headers(sq, q.codes, q.sl.nw_full, q.sl.full.bytes, q.sl.full);
    if (q.sl.T_tail)
      dmc::launch_write_headers(sq, q.codes + (size_t)q.sl.nw_full * q.sl.full.bytes, 1,
                                q.sl.tail.bytes, q.sl.tail);
    if (q.sl.nw_full)
      dmc::launch_autocorr(sq, q.frames, m.n, q.T, q.sl.nw_full, b->precision, shared,
                           (double*)(b->buf + q.o_R), q.P);
    if (q.sl.T_tail)
      dmc::launch_autocorr(sq, q.frames + (size_t)q.sl.nw_full * q.T * 3 * m.n * rs, m.n,
                           q.sl.T_tail, 1, b->precision, shared, (double*)(b->buf + q.o_Rt));
  }
  if ((e = batch_join(b, s, 0)) != hipSuccess) return e;
  if (!b->cs.empty() && (e = hipEventRecord(b->ev_fork[2], s)) != hipSuccess) return e;
  // the classes run side by side (each on its own stream when there are
  // branches); a sequence's second phase waits for its own classes only
  for (size_t c = 0; c < b->cls_n.size(); ++c) {
    hipStream_t sc = b->cs.empty() ? s : b->cs[c];
    if (!b->cs.empty() && (e = hipStreamWaitEvent(sc, b->ev_fork[2], 0)) != hipSuccess) return e;
    dmc::launch_oi_batch(sc, b->cls_tmax[c], b->cls_kr[c], b->precision,
                         (const dmc::OiArgs*)(b->buf + b->o_args),
                         (const int4*)(b->buf + b->o_jobs) + b->cls_off[c], b->cls_n[c]);
    if (!b->cs.empty() && (e = hipEventRecord(b->ev_cls[c], sc)) != hipSuccess) return e;
  }
  if ((e = batch_fork(b, s, 1)) != hipSuccess) return e;
  double* summary = (double*)(b->buf + b->o_summary);
  for (int i : b->order2) {
    BatchSeq& q = b->seq[i];
    const dmc::MeshDev& m = q.mesh->dev;
    hipStream_t sq = on(q);
    uint8_t* shared = shared_of(q);
    if (!b->cs.empty())
      for (int c : q.cls)
        if (c >= 0 && (e = hipStreamWaitEvent(sq, b->ev_cls[c], 0)) != hipSuccess) return e;
    if (q.sl.nw_full) {
      double* ud = (double*)(b->buf + q.o_ud);
      dmc::launch_dict_code(sq, (const double*)(b->buf + q.o_ut), q.sl.nw_full, q.sl.full,
                            q.codes, q.sl.full.bytes, ud);
      dmc::launch_project_quantise(sq, m, q.frames, q.T, q.k_full, q.sl.nw_full, b->precision,
                                   ud, q.codes, q.sl.full.bytes, q.sl.full, shared, nullptr);
      dmc::launch_anchors(sq, m, q.frames, q.T, q.sl.nw_full, b->precision, q.codes,
                          q.sl.full.bytes, q.sl.full, (double*)(b->buf + q.o_ap));
      dmc::launch_zero_tail(sq, q.codes, q.sl.nw_full, q.sl.full.bytes);
    }
    if (q.sl.T_tail) {
      const size_t f0 = (size_t)q.sl.nw_full * q.T;
      uint8_t* rec = q.codes + (size_t)q.sl.nw_full * q.sl.full.bytes;
      double* ud = (double*)(b->buf + q.o_udt);
      dmc::launch_dict_code(sq, (const double*)(b->buf + q.o_utt), 1, q.sl.tail, rec,
                            q.sl.tail.bytes, ud);
      dmc::launch_project_quantise(sq, m, q.frames + f0 * 3 * m.n * rs, q.sl.T_tail, q.k_tail,
                                   1, b->precision, ud, rec, q.sl.tail.bytes, q.sl.tail, shared,
                                   nullptr);
      dmc::launch_anchors(sq, m, q.frames + f0 * 3 * m.n * rs, q.sl.T_tail, 1, b->precision,
                          rec, q.sl.tail.bytes, q.sl.tail, (double*)(b->buf + q.o_apt));
      dmc::launch_zero_tail(sq, rec, 1, q.sl.tail.bytes);
    }
    if (q.out) {
      const DecodePlan d = decode_plan(m, q.sl, q.p);
      // the branches share the chip: a backward level needs a share of it
      decode_enqueue_fixed(sq, m, q.codes, q.sl, q.p, d, shared, q.out, q.p.cg_max_iters,
                           summary + 2 * i, b->br.empty() ? 2048 : 2048 / (int)b->br.size());
    }
  }
  return batch_join(b, s, 1);
}

// Branches of the batch's graph: independent sequences overlap on the GPU.
// Four, the HIP runtime's default number of hardware queues per process (on
// 64 sequences of 2k-60k vertices: 110 ms per run on one branch, 75 on two,
// 60 on four; eight branches ran no faster, and eight or sixteen hardware
// queues made the run slower).
int batch_branches(int32_t nseq) { return std::max(1, std::min<int>(4, nseq)); }

// Times `launch` (three runs after one warm-up) with events on stream s.
template <typename F>
float time_launch(hipStream_t s, F launch) {
  hipEvent_t a, z;
  if (hipEventCreate(&a) != hipSuccess) return 1e30f;
  if (hipEventCreate(&z) != hipSuccess) {
    (void)hipEventDestroy(a);
    return 1e30f;
  }
  launch();
  (void)hipEventRecord(a, s);
  for (int r = 0; r < 3; ++r) launch();
  (void)hipEventRecord(z, s);
  float ms = 1e30f;
  if (hipEventSynchronize(z) != hipSuccess || hipEventElapsedTime(&ms, a, z) != hipSuccess)
    ms = 1e30f;
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(z);
  return ms;
}

}  // namespace

dmc_status dmc_batch_create(dmc_ctx ctx, int32_t nseq, const dmc_mesh* meshes,
                            const void* const* frames, const int32_t* F, const int32_t* T,
                            const dmc_params* params, const void* const* q_start,
                            void* const* codes, void* const* frames_out, dmc_batch* out) {
  if (!ctx || !meshes || !frames || !F || !T || !params || !codes || !out)
    return fail(DMC_ERR_INVALID_ARG, "NULL argument");
  *out = nullptr;
  if (nseq < 1) return fail(DMC_ERR_INVALID_ARG, "nseq must be >= 1");
  HIP_TRY(hipSetDevice(ctx->device));
  auto b = new dmc_batch_s();
  b->ctx = ctx;
  b->precision = params[0].precision;
  auto bail = [&](dmc_status st) {
    delete b;
    return st;
  };
  Carve cv;
  size_t nargs = 0, njobs = 0, nwin = 0;
  std::vector<size_t> need(nseq);  // per sequence: bytes of its share of the branch scratch
  b->seq.resize(nseq);
  for (int32_t i = 0; i < nseq; ++i) {
    BatchSeq& q = b->seq[i];
    const dmc_params& p = params[i];
    dmc_status st = check_params(&p, T[i]);
    if (st != DMC_OK) return bail(st);
    if (!meshes[i] || meshes[i]->ctx != ctx || !frames[i] || !codes[i] || F[i] < 1)
      return bail(fail(DMC_ERR_INVALID_ARG, "sequence " + std::to_string(i) + ": bad argument"));
    if (p.precision != b->precision)
      return bail(fail(DMC_ERR_INVALID_ARG, "one precision per batch"));
    if (p.init == DMC_INIT_LEARNED)
      return bail(fail(DMC_ERR_UNSUPPORTED, "the learned start is not available in a batch"));
    const bool need_start = p.init == DMC_INIT_RANDOM || p.init == DMC_INIT_SKETCH;
    if (need_start && F[i] >= T[i] && (!q_start || !q_start[i]))
      return bail(fail(DMC_ERR_INVALID_ARG, "sequence " + std::to_string(i) + " needs q_start"));
    q.mesh = meshes[i];
    q.frames = (const uint8_t*)frames[i];
    q.F = F[i];
    q.T = T[i];
    q.p = p;
    q.q_start = q_start ? q_start[i] : nullptr;
    q.codes = (uint8_t*)codes[i];
    q.out = frames_out ? frames_out[i] : nullptr;
    const dmc::MeshDev& m = q.mesh->dev;
    q.sl = seq_layout(m.n, q.F, q.T, m.nc, p);
    q.k_full = std::min(p.k, q.T);
    q.k_tail = q.sl.T_tail ? std::min(p.k, q.sl.T_tail) : 0;
    q.o_R = cv.add((size_t)q.sl.nw_full * 3 * q.T * q.T * 8);
    q.o_ut = cv.add((size_t)q.sl.nw_full * 3 * q.T * q.k_full * 8);
    q.o_Rt = cv.add((size_t)3 * q.sl.T_tail * q.sl.T_tail * 8);
    q.o_utt = cv.add((size_t)3 * q.sl.T_tail * q.k_tail * 8);
    q.o_ud = cv.add((size_t)q.sl.nw_full * 3 * q.T * q.k_full * 8);
    q.o_udt = cv.add((size_t)3 * q.sl.T_tail * q.k_tail * 8);
    q.o_ap = cv.add(dmc::anchors_scratch_bytes(std::max(1, q.sl.nw_full)));
    q.o_apt = cv.add(dmc::anchors_scratch_bytes(1));
    q.stats_off = (int32_t)nwin;
    nwin += q.sl.nw_full + (q.sl.T_tail ? 1 : 0);
    // branch scratch: autocorrelation partials (any tuned split), projection
    // scratch and decoder buffers, used by one sequence at a time
    const int P0 = dmc::autocorr_blocks(m.n, std::max(1, q.sl.nw_full));
    const int Pmax = std::max(1, std::min(4 * P0, std::max(1, m.n)));
    need[i] = std::max(dmc::autocorr_scratch_bytes(m.n, q.T, std::max(1, q.sl.nw_full),
                                                   b->precision, Pmax),
                       dmc::project_scratch_bytes(m.n, q.T, q.k_full, std::max(1, q.sl.nw_full),
                                                  b->precision));
    if (q.out) need[i] = std::max(need[i], decode_plan(m, q.sl, p).lay.total);
    if (q.sl.nw_full) {
      ++nargs;
      njobs += p.init == DMC_INIT_PREV ? 3 : 3 * (size_t)q.sl.nw_full;
    }
    if (q.sl.T_tail) {
      ++nargs;
      njobs += 3;
    }
  }
  // sequences to branches, largest first onto the least loaded (vertex-frames)
  const int nbranch = batch_branches(nseq);
  {
    std::vector<int> order(nseq);
    for (int32_t i = 0; i < nseq; ++i) order[i] = i;
    auto work = [&](int i) { return (double)b->seq[i].mesh->dev.n * b->seq[i].F; };
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return work(x) > work(y); });
    std::vector<double> load(nbranch, 0.0);
    std::vector<size_t> bytes(nbranch, 0);
    for (int i : order) {
      const int j = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      b->seq[i].branch = j;
      load[j] += work(i);
      bytes[j] = std::max(bytes[j], need[i]);
    }
    for (int j = 0; j < nbranch; ++j) b->o_shared.push_back(cv.add(bytes[j]));
  }
  b->o_args = cv.add(nargs * sizeof(dmc::OiArgs));
  b->o_jobs = cv.add(njobs * sizeof(int4));
  b->o_summary = cv.add((size_t)nseq * 2 * sizeof(double));
  b->o_stats = cv.add(nwin * sizeof(dmc::StatsDev));
  if (hipMalloc(&b->buf, cv.total()) != hipSuccess) {
    (void)hipGetLastError();
    return bail(fail(DMC_ERR_OUT_OF_MEMORY, "cannot allocate the batch's scratch"));
  }
  // orthogonal-iteration arguments and jobs, grouped into launch classes
  std::vector<dmc::OiArgs> args;
  std::vector<std::array<int, 6>> jobs;  // tmax, kr, args index, w0, w1, c
  dmc::StatsDev* stats = (dmc::StatsDev*)(b->buf + b->o_stats);
  for (BatchSeq& q : b->seq) {
    for (int part = 0; part < 2; ++part) {
      const bool tail = part == 1;
      const int32_t nw = tail ? (q.sl.T_tail ? 1 : 0) : q.sl.nw_full;
      if (!nw) continue;
      dmc::OiArgs a{};
      a.R = (const double*)(b->buf + (tail ? q.o_Rt : q.o_R));
      a.nw = nw;
      a.T = tail ? q.sl.T_tail : q.T;
      a.k = tail ? q.k_tail : q.k_full;
      a.precision = b->precision;
      a.init = tail ? DMC_INIT_EXACT : q.p.init;
      a.ncoord = 3;
      a.q_start = (tail || q.p.init == DMC_INIT_EXACT) ? nullptr : q.q_start;
      a.q_learned = nullptr;
      a.u_out = nullptr;
      a.u_canon = (double*)(b->buf + (tail ? q.o_utt : q.o_ut));
      a.max_sweeps = q.p.oi_max_sweeps;
      a.tol = q.p.oi_tol;
      a.stats = stats + q.stats_off + (tail ? q.sl.nw_full : 0);
      const int ai = (int)args.size();
      args.push_back(a);
      const int tmax = a.T <= 32 ? 32 : 64, kr = a.k <= 16 ? 16 : 32;
      for (int c = 0; c < 3; ++c) {
        if (a.init == DMC_INIT_PREV)
          jobs.push_back({tmax, kr, ai, 0, nw, c});
        else
          for (int w = 0; w < nw; ++w) jobs.push_back({tmax, kr, ai, w, w + 1, c});
      }
    }
  }
  std::stable_sort(jobs.begin(), jobs.end(), [](const std::array<int, 6>& x,
                                                const std::array<int, 6>& y) {
    return x[0] != y[0] ? x[0] < y[0] : x[1] < y[1];
  });
  std::vector<int4> dj(jobs.size());
  for (size_t j = 0; j < jobs.size(); ++j) {
    dj[j] = make_int4(jobs[j][2], jobs[j][3], jobs[j][4], jobs[j][5]);
    if (j == 0 || jobs[j][0] != jobs[j - 1][0] || jobs[j][1] != jobs[j - 1][1]) {
      b->cls_tmax.push_back(jobs[j][0]);
      b->cls_kr.push_back(jobs[j][1]);
      b->cls_off.push_back((int)j);
      b->cls_n.push_back(0);
    }
    ++b->cls_n.back();
  }
  // each sequence's classes, and the second phase's order: sequences whose
  // slowest class is the cheapest first (its windows' T and k bound a class's
  // time), so a branch works on them while the larger classes still run
  auto class_of = [&](int T, int k) {
    const int tmax = T <= 32 ? 32 : 64, kr = k <= 16 ? 16 : 32;
    for (size_t c = 0; c < b->cls_n.size(); ++c)
      if (b->cls_tmax[c] == tmax && b->cls_kr[c] == kr) return (int)c;
    return -1;
  };
  std::vector<int> slowest(nseq, 0);
  for (int32_t i = 0; i < nseq; ++i) {
    BatchSeq& q = b->seq[i];
    if (q.sl.nw_full) q.cls[0] = class_of(q.T, q.k_full);
    if (q.sl.T_tail) q.cls[1] = class_of(q.sl.T_tail, q.k_tail);
    for (int c : q.cls)
      if (c >= 0) slowest[i] = std::max(slowest[i], b->cls_tmax[c] * b->cls_kr[c]);
    b->order2.push_back(i);
  }
  std::stable_sort(b->order2.begin(), b->order2.end(),
                   [&](int x, int y) { return slowest[x] < slowest[y]; });
  if (hipMemcpy(b->buf + b->o_args, args.data(), args.size() * sizeof(dmc::OiArgs),
                hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(b->buf + b->o_jobs, dj.data(), dj.size() * sizeof(int4),
                hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipFree(b->buf);
    return bail(fail(DMC_ERR_DEVICE, "cannot upload the batch's job table"));
  }
  // autotuner: vertex split of the covariance kernel, timed on each
  // sequence's own frames
  hipStream_t s = ctx->stream;
  for (BatchSeq& q : b->seq) {
    const dmc::MeshDev& m = q.mesh->dev;
    if (!q.sl.nw_full) continue;
    uint8_t* sh = b->buf + b->o_shared[q.branch];
    const int P0 = dmc::autocorr_blocks(m.n, q.sl.nw_full);
    float best = 1e30f;
    for (int P : {P0 / 4, P0 / 2, P0, 2 * P0, 4 * P0}) {
      if (P < 1 || P > std::max(1, m.n)) continue;
      const float t = time_launch(s, [&] {
        dmc::launch_autocorr(s, q.frames, m.n, q.T, q.sl.nw_full, b->precision, sh,
                             (double*)(b->buf + q.o_R), P);
      });
      if (t < best) {
        best = t;
        q.P = P;
      }
    }
  }
  dmc_status st = check_launch("batch autotuner");
  bool ok = st == DMC_OK &&
            hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) == hipSuccess &&
            hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming) == hipSuccess &&
            hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming) == hipSuccess;
  if (ok && nbranch > 1) {
    b->br.assign(nbranch, nullptr);
    b->cs.assign(b->cls_n.size(), nullptr);
    b->ev_fork.assign(3, nullptr);
    b->ev_join.assign(2 * nbranch, nullptr);
    b->ev_cls.assign(b->cls_n.size(), nullptr);
    for (hipStream_t& x : b->br)
      ok = ok && hipStreamCreateWithFlags(&x, hipStreamNonBlocking) == hipSuccess;
    for (hipStream_t& x : b->cs)
      ok = ok && hipStreamCreateWithFlags(&x, hipStreamNonBlocking) == hipSuccess;
    for (hipEvent_t& x : b->ev_cls)
      ok = ok && hipEventCreateWithFlags(&x, hipEventDisableTiming) == hipSuccess;
    for (hipEvent_t& x : b->ev_fork)
      ok = ok && hipEventCreateWithFlags(&x, hipEventDisableTiming) == hipSuccess;
    for (hipEvent_t& x : b->ev_join)
      ok = ok && hipEventCreateWithFlags(&x, hipEventDisableTiming) == hipSuccess;
  }
  if (st == DMC_OK && !ok) {
    (void)hipGetLastError();
    st = fail(DMC_ERR_DEVICE, "cannot create the batch's streams");
  }
  if (st != DMC_OK) {
    dmc_batch_destroy(b);
    return st;
  }
  *out = b;
  return DMC_OK;
}

dmc_status dmc_batch_run(dmc_batch b) {
  if (!b) return fail(DMC_ERR_INVALID_ARG, "NULL batch");
  HIP_TRY(hipSetDevice(b->ctx->device));
  hipStream_t s = b->stream;
  if (!b->exec) {
    dmc::prof::pause(true);
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      const hipError_t e1 = batch_enqueue(b, s);
      e = hipStreamEndCapture(s, &b->graph);
      if (e1 != hipSuccess) {
        if (e == hipSuccess) (void)hipGraphDestroy(b->graph);
        b->graph = nullptr;
        e = e1;
      }
    }
    dmc::prof::pause(false);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(DMC_ERR_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    }
    HIP_TRY(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  }
  // ordered after earlier work on the context's stream, and before later work
  HIP_TRY(hipEventRecord(b->ev_in, b->ctx->stream));
  HIP_TRY(hipStreamWaitEvent(s, b->ev_in, 0));
  HIP_TRY(hipGraphLaunch(b->exec, s));
  HIP_TRY(hipEventRecord(b->ev_out, s));
  HIP_TRY(hipStreamWaitEvent(b->ctx->stream, b->ev_out, 0));
  return check_launch("batch graph");
}

dmc_status dmc_batch_stats(dmc_batch b, int32_t i, dmc_window_stats* per_window) {
  if (!b || !per_window) return fail(DMC_ERR_INVALID_ARG, "NULL argument");
  if (i < 0 || i >= (int32_t)b->seq.size()) return fail(DMC_ERR_INVALID_ARG, "bad sequence index");
  const BatchSeq& q = b->seq[i];
  const int32_t nw = q.sl.nw_full + (q.sl.T_tail ? 1 : 0);
  HIP_TRY(hipSetDevice(b->ctx->device));
  dmc_status st = ensure_pinned(b->ctx, sizeof(dmc::StatsDev) * nw + 64);
  if (st != DMC_OK) return st;
  uint8_t* h = (uint8_t*)b->ctx->pinned;
  HIP_TRY(hipMemcpyAsync(h, b->buf + b->o_stats + q.stats_off * sizeof(dmc::StatsDev),
                         sizeof(dmc::StatsDev) * nw, hipMemcpyDeviceToHost, b->ctx->stream));
  HIP_TRY(hipMemcpyAsync(h + sizeof(dmc::StatsDev) * nw, b->buf + b->o_summary + 16 * i, 16,
                         hipMemcpyDeviceToHost, b->ctx->stream));
  HIP_TRY(hipStreamSynchronize(b->ctx->stream));
  std::vector<dmc::StatsDev> hs((const dmc::StatsDev*)h, (const dmc::StatsDev*)h + nw);
  double sum[2];
  std::memcpy(sum, h + sizeof(dmc::StatsDev) * nw, sizeof(sum));
  std::vector<std::vector<uint8_t>> heads;
  st = read_record_heads(b->ctx, q.codes, q.sl.nw_full, q.sl.full,
                         q.sl.T_tail ? &q.sl.tail : nullptr, heads);
  if (st != DMC_OK) return st;
  for (int32_t w = 0; w < nw; ++w) {
    std::memset(&per_window[w], 0, sizeof(dmc_window_stats));
    const bool tail = w >= q.sl.nw_full;
    fill_stats(&per_window[w], hs[w], tail ? q.sl.tail : q.sl.full, heads[w].data());
    per_window[w].cg_iters = q.out ? q.p.cg_max_iters : 0;
    per_window[w].cg_resid = q.out ? sum[0] : 0.0;
  }
  if (q.out && sum[1] == 0.0)
    return fail(DMC_ERR_NOT_CONVERGED, "sequence " + std::to_string(i) +
                                           ": some column did not reach cg_tol");
  if (oi_not_converged(hs.data(), nw, q.p.oi_tol))
    return fail(DMC_ERR_NOT_CONVERGED, "sequence " + std::to_string(i) +
                                           ": orthogonal iterations ended above oi_tol");
  return DMC_OK;
}

dmc_status dmc_batch_tuning(dmc_batch b, int32_t i, int32_t tuning[2]) {
  if (!b || !tuning) return fail(DMC_ERR_INVALID_ARG, "NULL argument");
  if (i < 0 || i >= (int32_t)b->seq.size()) return fail(DMC_ERR_INVALID_ARG, "bad sequence index");
  tuning[0] = b->seq[i].P;
  tuning[1] = b->seq[i].branch;
  return DMC_OK;
}

void dmc_batch_destroy(dmc_batch b) {
  if (!b) return;
  (void)hipSetDevice(b->ctx->device);
  (void)hipStreamSynchronize(b->ctx->stream);
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->ev_in) (void)hipEventDestroy(b->ev_in);
  if (b->ev_out) (void)hipEventDestroy(b->ev_out);
  for (hipEvent_t x : b->ev_fork)
    if (x) (void)hipEventDestroy(x);
  for (hipEvent_t x : b->ev_join)
    if (x) (void)hipEventDestroy(x);
  for (hipEvent_t x : b->ev_cls)
    if (x) (void)hipEventDestroy(x);
  for (hipStream_t x : b->br)
    if (x) (void)hipStreamDestroy(x);
  for (hipStream_t x : b->cs)
    if (x) (void)hipStreamDestroy(x);
  if (b->stream) (void)hipStreamDestroy(b->stream);
  if (b->buf) (void)hipFree(b->buf);
  delete b;
}
