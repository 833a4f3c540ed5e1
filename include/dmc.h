/*
 * dmc.h -- C ABI of the MI355X (gfx950) spatio-temporal dynamic-mesh compressor.
 *
 * Method: Arvanitis, Lalos, Moustakas, "Fast Spatio-temporal Compression of
 * Dynamic 3D Meshes" (arXiv 2111.10105).  Per window of T consecutive frames of
 * a mesh with fixed connectivity (Sec. II, Sec. III-A) the encoder computes
 *   delta coordinates     delta = L V for every frame          (Eq. 3-4, Eq. 8)
 *   autocorrelation       R_c = A_c A_c^T, c in {x, y, z}       (Eq. 7)
 *   eigen-trajectories    first k eigenvectors of R_c, by orthogonal
 *                         iterations warm-started from the previous window
 *                         (Algorithm 1) and a Rayleigh-Ritz step  (Eq. 5)
 *   coefficients          Y_c = U_k^T delta_c^T                 (Eq. 9)
 *   codes                 uniform quantisation of the k rows     (Eq. 10)
 *   anchors               quantised coordinates of the vertices in N (Eq. 12)
 * and the decoder solves the anchored least-squares system of Eq. (12) for all
 * frames at once, by conjugate gradients on its normal equations
 * (L^T L + I_N^T I_N) X = L^T (U Y) ^T + I_N^T A_N.
 *
 * Conventions (every entry point):
 *  - Pointers named *_dev are device pointers (HIP); *_host are host pointers.
 *    The caller owns every buffer it passes; the library never frees them.
 *  - Scratch memory: by default the context allocates its kernels' scratch on
 *    first use, grows it when a call needs more and keeps it until
 *    dmc_destroy.  A caller that must not allocate gives a workspace instead
 *    (dmc_set_workspace, sized by dmc_workspace_bytes): then encode and
 *    decode calls allocate nothing and fail with DMC_ERR_BUFFER_TOO_SMALL
 *    when the workspace is short.  The context also owns small stats and
 *    staging buffers made by dmc_create, and the meshes made with it.
 *  - All device work is ordered on the context's HIP stream.  The encode,
 *    decode and sequence calls synchronise it once at their end (they read
 *    convergence flags there); the single-step and learned-start calls
 *    return after enqueueing.
 *  - Errors are returned as dmc_status, never by aborting; dmc_last_error()
 *    gives a message for the calling thread.  Arguments are validated on the
 *    host before any launch; on error no output is written.
 *  - Frames are float64 when params.precision == DMC_FP64, else float32, laid
 *    out [frame][vertex][xyz] (row-major, xyz interleaved).
 */
#ifndef DMC_H
#define DMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dmc_ctx_s* dmc_ctx;
typedef struct dmc_mesh_s* dmc_mesh;

typedef enum {
  DMC_OK = 0,
  DMC_ERR_INVALID_ARG = 1,
  DMC_ERR_OUT_OF_MEMORY = 2,
  DMC_ERR_DEVICE = 3,
  DMC_ERR_NOT_CONVERGED = 4,
  DMC_ERR_SINGULAR = 5,
  DMC_ERR_BUFFER_TOO_SMALL = 6,
  DMC_ERR_UNSUPPORTED = 7
} dmc_status;

/* arithmetic of the encoder's GEMMs (frames dtype follows: FP64 -> double,
 * otherwise float).  DMC_BF16 is the precision form: float32 frames; the
 * covariance (Eq. 7) and the C.Q products of the orthogonal iterations take
 * bfloat16 operands with float32 accumulation on the matrix cores; the
 * iterations run with those products to a stage tolerance
 * (DMC_BF16_STAGE_TOL, or oi_tol if larger), then refine with
 * full-precision products (at least one sweep) until oi_tol, or until a
 * sweep reduces the residual by less than a tenth (the bfloat16 covariance
 * fixes its small eigen-directions only to its own rounding, and there the
 * iterations stall); the k x k Cholesky factors and the Ritz eigen-solve
 * stay float64; everything else is as DMC_FP32. */
enum { DMC_FP64 = 0, DMC_FP32 = 1, DMC_BF16 = 2 };
#define DMC_BF16_STAGE_TOL 3e-2

/* Laplacian: Eq. (3) I - D^-1 C (default) or Eq. (1) D - C */
enum { DMC_LAP_UNIFORM = 0, DMC_LAP_COMBINATORIAL = 1 };

/* preconditioner of the decoder's conjugate gradients: none, the diagonal of
 * the normal matrix, or its sparse Cholesky factor (computed once per mesh by
 * dmc_mesh_create) */
enum { DMC_PRECOND_NONE = 0, DMC_PRECOND_JACOBI = 1, DMC_PRECOND_CHOLESKY = 2 };

/* start block of each window's orthogonal iterations (Algorithm 1):
 * DMC_INIT_PREV   the previous window's U_k (Algorithm 1's warm start); window 0
 *                 from q_start [3][T][k], or its exact eigenvectors (Eq. 5)
 *                 if q_start is NULL.  Windows run in order.
 * DMC_INIT_RANDOM a caller-given block per window, q_start [nw][3][T][k]
 *                 (e.g. seeded Gaussian); windows run concurrently.
 * DMC_INIT_SKETCH the sketch R_c Omega of each window with one caller-given
 *                 q_start = Omega [T][k] for all windows and coordinates;
 *                 windows run concurrently.
 * DMC_INIT_EXACT  every window from its exact eigenvectors (Eq. 5, the
 *                 per-block SVD); q_start is ignored; windows run concurrently.
 * DMC_INIT_LEARNED the network registered with dmc_learned_start predicts
 *                 each window's start from its sketch R_c Omega; windows run
 *                 concurrently; q_start is ignored.
 * Start blocks are in the frames' type.  A shorter last window of a sequence
 * always starts from its exact eigenvectors. */
enum { DMC_INIT_PREV = 0, DMC_INIT_RANDOM = 1, DMC_INIT_SKETCH = 2, DMC_INIT_EXACT = 3,
       DMC_INIT_LEARNED = 4 };

typedef struct {
  int32_t k;             /* kept rows k_l of Eq. (10), 1 <= k <= T            */
  int32_t coef_bits;     /* bits of Q(.) in Eq. (10): 1..16, 0 = raw values    */
  int32_t anchor_bits;   /* bits per anchor coordinate: 1..16, 0 = raw values  */
  int32_t dict_bits;     /* bits per dictionary entry:  1..16, 0 = raw values  */
  int32_t precision;     /* DMC_FP64, DMC_FP32 or DMC_BF16                     */
  int32_t oi_max_sweeps; /* cap on orthogonal-iteration sweeps per window >= 1
                            (>= 2 for DMC_BF16)                                */
  double oi_tol;         /* stop when ||R Q - Q Q^T R Q||_F <= tol ||R||_F     */
  int32_t cg_max_iters;  /* cap on conjugate-gradient iterations >= 1          */
  int32_t precond;       /* DMC_PRECOND_*                                      */
  double cg_tol;         /* stop a column when ||r|| <= tol ||b||              */
  int32_t init;          /* DMC_INIT_* (0 = DMC_INIT_PREV, Algorithm 1)        */
  int32_t dict_mode;     /* DMC_DICT_PLAIN (0) or DMC_DICT_ADAPTIVE (1)        */
  double coef_step;      /* 0: coef_bits for every kept row (Eq. 10); > 0: each
                            row takes the fewest bits <= coef_bits whose step
                            (hi - lo) / (2^b - 1) is at most coef_step        */
} dmc_params;

/* Dictionary coding (Sec. IV).  DMC_DICT_PLAIN: every entry of U_k coded with
 * dict_bits over [-1, 1].  DMC_DICT_ADAPTIVE: each column of a window's U_k
 * coded over its own range (float32, rounded outwards), either as its values
 * or as its difference from the same column of the previous window's
 * dequantised dictionary in the same sequence (the block-to-block coding the
 * paper describes with Fig. 6), whichever needs fewer bits, with the fewest
 * bits whose step is at most 2 / (2^dict_bits - 1), the plain code's; so no
 * entry is coded less precisely than in the plain form.  A sequence's first
 * window, and any window after one of another length, uses values only. */
enum { DMC_DICT_PLAIN = 0, DMC_DICT_ADAPTIVE = 1 };

/* Per-window statistics.  The bit rates follow Eq. (13) read per coordinate:
 * bits of the window's record part divided by 3 n T (vertices x frames x
 * coordinates): q the coefficient codes of Eq. (10) with their row ranges,
 * q_a the anchor codes with their range, q_d the dictionary, q_s = q + q_a +
 * q_d.  ms_encode and ms_decode are the stream times of the whole call's
 * encode and decode (the same in every window's entry of a sequence call). */
typedef struct {
  int32_t T, k;             /* window length and kept rows                     */
  int32_t oi_sweeps[3];     /* sweeps per coordinate (0 = exact start)         */
  double oi_resid[3];       /* final ||RQ - QH||_F / ||R||_F per coordinate    */
  int32_t chol_shifts[3];   /* CholeskyQR breakdowns repaired by a shift       */
  int32_t cg_iters;         /* decoder iterations (0 if not decoded)           */
  double cg_resid;          /* max over columns of ||r|| / ||b||               */
  double q, q_a, q_d, q_s;  /* bits per vertex per frame and coordinate        */
  float ms_encode, ms_decode;
} dmc_window_stats;

/* ---- context -------------------------------------------------------------
 * dmc_create: bind to HIP device `device`; `hip_stream` is a hipStream_t (NULL
 * = the legacy default stream).  DMC_ERR_DEVICE if the device is not a
 * gfx950 GPU or cannot be used. */
dmc_status dmc_create(int32_t device, void* hip_stream, dmc_ctx* out);
void dmc_destroy(dmc_ctx ctx);
dmc_status dmc_set_stream(dmc_ctx ctx, void* hip_stream);
const char* dmc_last_error(void);
/* bytes of scratch the context has allocated itself (0 while a caller's
 * workspace is in use) */
size_t dmc_scratch_bytes(dmc_ctx ctx);
/* dmc_workspace_bytes: device bytes of scratch that dmc_compress_sequence
 * (with or without decoding) and dmc_decode_sequence need for F frames in
 * windows of T on this mesh with these params; with F = T, the same for
 * dmc_encode_window and dmc_decode_window.  0 for invalid arguments.
 * dmc_set_workspace: the context uses dev_ptr [bytes] (device memory owned
 * by the caller, 256-byte aligned, kept alive and unused by the caller until
 * it is replaced or the context destroyed) as its scratch and frees any
 * scratch it allocated itself; NULL and 0 return to library-allocated
 * scratch.  Synchronises the context's stream.  With a workspace set, a call
 * that needs more returns DMC_ERR_BUFFER_TOO_SMALL before launching. */
size_t dmc_workspace_bytes(dmc_mesh mesh, int32_t F, int32_t T, const dmc_params* params);
dmc_status dmc_set_workspace(dmc_ctx ctx, void* dev_ptr, size_t bytes);

/* ---- mesh (Sec. II) ------------------------------------------------------
 * Builds, once per mesh, the binary adjacency C of Eq. (2) (edges of the
 * triangles, duplicates merged), the degrees d_i, the Laplacian chosen by
 * `laplacian`, and the normal matrix L^T L + I_N^T I_N of Eq. (12), and copies
 * them to the device.  tris_host: int32 [n_tris][3]; anchors_host: int32
 * [n_anchors], distinct vertex indices (the set N of Eq. 12; anchor values are
 * stored in this order).  Errors: DMC_ERR_INVALID_ARG for an index out of
 * range, a repeated anchor, or a vertex with no neighbour (Eq. 3 undefined);
 * DMC_ERR_SINGULAR when a connected component holds no anchor.  The sparse
 * Cholesky factor of the normal matrix (the decoder's preconditioner) is
 * ordered and analysed on the host (nested dissection, supernodes) and
 * factorised on the device, level by level of the supernodal tree.
 * Synchronises the context's stream. */
dmc_status dmc_mesh_create(dmc_ctx ctx, int32_t n_verts, int32_t n_tris,
                           const int32_t* tris_host, int32_t n_anchors,
                           const int32_t* anchors_host, int32_t laplacian,
                           dmc_mesh* out);
void dmc_mesh_destroy(dmc_mesh mesh);
int32_t dmc_mesh_nnz(dmc_mesh mesh);          /* nonzeros of C (= 2 |E|)       */
int32_t dmc_mesh_normal_nnz(dmc_mesh mesh);   /* nonzeros of L^T L + I_N^T I_N */
/* sizes of the normal matrix's Cholesky factor, DMC_FACTOR_INFO_LEN values:
 * [0] stored entries, [1] nonzeros of the exact factor, [2] supernodes,
 * [3] tree levels, [4] factorisation flops, [5] seconds to build the factor
 * (host ordering and symbolic analysis, then the numeric factorisation and
 * the solve operators on the device; all on the host for
 * dmc_host_normal_solve),
 * [6] entries of the solve operators one triangular solve reads (per
 * right-hand side: 2 flops each), [7] update rows (entries of the factor left
 * of a diagonal block, counted by row of the supernode that produces them),
 * [8] columns of the leaf supernodes (rows the forward solve takes straight
 * from the right-hand side: no update reaches them) */
#define DMC_FACTOR_INFO_LEN 9
void dmc_mesh_factor_info(dmc_mesh mesh, double info[DMC_FACTOR_INFO_LEN]);
/* Whether the mesh holds its anchor response G = (L^T L + I_N^T I_N)^{-1}
 * I_N^T (n x n_c, float64 on the device).  The right-hand side of Eq. (12) is
 * linear in the decoded delta coordinates and anchor values, so with G the
 * decoder can solve the 3k columns L^T Y^^T of each window instead of its 3T
 * frames' columns and form X = Z U~^T + G A^ (same solution up to rounding).
 * Cost model: a solved column costs S = 16 x (entries of the solve operators,
 * dmc_mesh_factor_info [6]), the product A = 2 n n_c per output column.
 * dmc_mesh_create builds G when 2 A <= S and it takes at most 2 GiB; a decode
 * uses it when nz S + 3F A < 3F S (nz the reduced columns).  The convergence
 * test then bounds the relative residual of every frame's full system of
 * Eq. (12) by cg_tol, counting G's own residual.  Returns 1 if built
 * and writes, where the pointers are not NULL, the conjugate-gradient
 * iterations of its solve and the largest relative residual of its columns;
 * 0 if not built (the decoder then solves 3T columns per window) or for a
 * NULL mesh. */
int32_t dmc_mesh_anchor_response(dmc_mesh mesh, int32_t* cg_iters, double* resid);

/* Solves (L^T L + I_N^T I_N) X = B, the normal matrix of Eq. (12), for
 * ncols right-hand sides with the mesh's sparse Cholesky factor (the
 * decoder's preconditioner, factorised on the device by dmc_mesh_create):
 * one forward and one backward supernodal solve, no iteration.  B_dev and
 * X_dev are float64 [n][ncols] row-major device arrays in vertex order and
 * may not alias.  Uses the context's scratch, or its workspace
 * (DMC_ERR_BUFFER_TOO_SMALL when that is short).  Synchronises the context's
 * stream at the end. */
dmc_status dmc_mesh_normal_solve(dmc_ctx ctx, dmc_mesh mesh, int32_t ncols, const double* B_dev,
                                 double* X_dev);

/* Host-only check of the ordering and factorisation (no device needed):
 * builds L^T L + I_N^T I_N and its supernodal Cholesky factor exactly as
 * dmc_mesh_create does, then solves (L^T L + I_N^T I_N) X = B on the host with
 * the same blocked algorithm the device uses.  B and X are float64
 * [n][ncols] row-major host arrays (may alias).  Same errors as
 * dmc_mesh_create. */
dmc_status dmc_host_normal_solve(int32_t n_verts, int32_t n_tris, const int32_t* tris_host,
                                 int32_t n_anchors, const int32_t* anchors_host,
                                 int32_t laplacian, int32_t ncols, const double* B_host,
                                 double* X_host, double info[DMC_FACTOR_INFO_LEN]);

/* ---- encoded window record -----------------------------------------------
 * One window's record is a byte buffer (device memory) of
 * dmc_window_code_bytes bytes (its capacity); its stream is its first
 * "used" bytes (header words 11-12), all defined, the rest of the slot zero.
 *   header   128 B: int32 words 0 magic "DMC2", 1 T, 2 k, 3 n, 4 n_c,
 *            5 coef_bits, 6 anchor_bits, 7 dict_bits, 8 precision,
 *            9 dict_mode, 10 1 if some dictionary column is a difference
 *            from the previous window's, 11-12 used bytes (low, high),
 *            13 words of the dictionary segments, 14-15 coef_step (double);
 *            the rest zero.
 *   tables   [3][k] dictionary columns, then [3][k] coefficient rows (row
 *            r of coordinate c at index c k + r), 16 B each: float32 lo, hi;
 *            uint32 bits (low byte) | mode << 8 (columns: 0 values, 1
 *            difference); uint32 first 32-bit word of the segment in the
 *            variable part.  Then the anchor ranges [3][2] float32.
 *   anchors  from the next 256-byte boundary: [3] segments of T n_c codes
 *            (index t n_c + a) at anchor_bits.
 *   variable from the next 256-byte boundary: every dictionary column's
 *            segment (T codes), then every coefficient row's (n codes), back
 *            to back at the offsets of the tables.
 * A segment holds codes of b bits packed least significant bit first (code
 * j in bits [j b, (j + 1) b) of the segment's bit string, bit i of which is
 * bit i mod 32 of 32-bit word i / 32), zero-padded to a multiple of 8 bytes;
 * with bits = 0 (coef_bits, anchor_bits or dict_bits 0) it holds raw values
 * (float64 for DMC_FP64, else float32).  A code c over [lo, hi] with b bits
 * stands for lo + c (hi - lo) / (2^b - 1); a row or column of 0 bits stands
 * for lo everywhere (hi = lo).  The plain dictionary code has lo = -1, hi =
 * 1 and dict_bits bits.  A record is self-contained given the mesh
 * (connectivity and N are side information shared with the decoder, as in
 * Sec. III), except that a difference column needs the previous window's
 * record of the same sequence. */
size_t dmc_window_code_bytes(int32_t n, int32_t T, int32_t n_anchors,
                             const dmc_params* params);
/* sum of dmc_window_code_bytes over the windows of an F-frame sequence */
size_t dmc_sequence_code_bytes(int32_t n, int32_t F, int32_t T, int32_t n_anchors,
                               const dmc_params* params);

/* ---- encode one window (Eq. 3-10, Eq. 12 anchors; Algorithm 1) -----------
 * frames_dev  [T][n][3] frames of the window.
 * q_start_dev start of the orthogonal iterations: with DMC_INIT_PREV or
 *             DMC_INIT_RANDOM a [3][T][k] block per coordinate (normally the
 *             previous window's u_out, the warm start of Algorithm 1), or NULL
 *             for the exact eigenvectors of R_c (Eq. 5); with
 *             DMC_INIT_SKETCH Omega [T][k] (start R_c Omega); ignored with
 *             DMC_INIT_EXACT.
 * code_dev    record buffer of dmc_window_code_bytes bytes.
 * u_out_dev   optional [3][T][k]: the window's eigen-trajectories U_k (before
 *             dictionary quantisation), columns ordered by eigenvalue,
 *             largest first, sign fixed so each column's largest-magnitude
 *             entry is positive.
 * coef_out_dev optional [3][k][n]: the coefficients Y of Eq. (9) before
 *             quantisation (computed with the dequantised dictionary).
 * stats       optional.
 * Synchronises the stream at its end and returns DMC_ERR_NOT_CONVERGED
 * (outputs still written) if the orthogonal iterations of some coordinate
 * ended with a residual above oi_tol, at oi_max_sweeps or where the precision
 * form's refinement stopped improving; an exact start is not iterated and
 * never reports it. */
dmc_status dmc_encode_window(dmc_ctx ctx, dmc_mesh mesh, const void* frames_dev,
                             int32_t T, const dmc_params* params,
                             const void* q_start_dev, void* code_dev,
                             void* u_out_dev, void* coef_out_dev,
                             dmc_window_stats* stats);

/* ---- encode one window without allocating --------------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * operation, arguments, outputs and errors as dmc_encode_window, bit for bit
 * the same results, but its scratch (delta coordinates, autocorrelation
 * partials, covariance, dictionary, coefficients and the window's stats)
 * lives in a fixed device array of the library of DMC_NOALLOC_SCRATCH_BYTES
 * per GPU, held from the first dmc_create on that GPU until the process
 * ends.  A window that needs more returns DMC_ERR_BUFFER_TOO_SMALL before
 * launching (its need is about T n (3 x frame bytes + 3 k x frame bytes) plus
 * the autocorrelation partials; e.g. 16,384 vertices x 32 frames fits).
 * Nothing is allocated by the call; it synchronises the stream at its end
 * like dmc_encode_window.  Every call on one GPU shares that GPU's array and
 * each call writes all of it that it reads: calls that overlap in time on
 * one GPU (two streams, two threads) race and must be serialised by the
 * caller. */
#define DMC_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
dmc_status dmc_encode_window_noalloc(dmc_ctx ctx, dmc_mesh mesh, const void* frames_dev,
                                     int32_t T, const dmc_params* params,
                                     const void* q_start_dev, void* code_dev, void* u_out_dev,
                                     void* coef_out_dev, dmc_window_stats* stats);

/* ---- decode one window (Eq. 12) ------------------------------------------
 * code_dev: a record written by dmc_encode_window for this mesh and T;
 * frames_out_dev [T][n][3].  The record's header is read back first: a
 * magic, T, k, n, n_c, bit widths or precision that differ from the call's
 * give DMC_ERR_INVALID_ARG before any kernel runs.  DMC_ERR_NOT_CONVERGED if
 * some column did not reach cg_tol within cg_max_iters (the last iterate is
 * still written). */
dmc_status dmc_decode_window(dmc_ctx ctx, dmc_mesh mesh, const void* code_dev,
                             int32_t T, const dmc_params* params,
                             void* frames_out_dev, dmc_window_stats* stats);

/* ---- whole sequence (Sec. III-A, "blocks") -------------------------------
 * Splits F frames into windows of T (the last may be shorter) and encodes
 * them, each window's orthogonal iterations starting as params->init says
 * (DMC_INIT_PREV: in order, from the previous window's U_k, window 0 from
 * q_start_dev [3][T][k] or exact if NULL; DMC_INIT_RANDOM: q_start_dev
 * [nw][3][T][k] for the nw = F / T full windows; DMC_INIT_SKETCH: Omega
 * [T][k]), writing the records back to back into codes_dev
 * (dmc_sequence_code_bytes bytes).  If frames_out_dev [F][n][3] is not NULL,
 * then decodes every window in one solve: over the 3k columns L^T Y^^T of
 * each window when the mesh holds its anchor response and the cost rule of
 * dmc_mesh_anchor_response picks that form, else over all 3F frame columns.
 * per_window: optional array of n_windows stats.  Synchronises once at the
 * end; DMC_ERR_NOT_CONVERGED (outputs still written) if the decoder's
 * conjugate gradients or some window's orthogonal iterations did not reach
 * their tolerance (as for dmc_encode_window). */
dmc_status dmc_compress_sequence(dmc_ctx ctx, dmc_mesh mesh, const void* frames_dev,
                                 int32_t F, int32_t T, const dmc_params* params,
                                 const void* q_start_dev, void* codes_dev,
                                 size_t codes_bytes, void* frames_out_dev,
                                 dmc_window_stats* per_window);

/* decode every record of a sequence written by dmc_compress_sequence; the
 * headers are checked as in dmc_decode_window */
dmc_status dmc_decode_sequence(dmc_ctx ctx, dmc_mesh mesh, const void* codes_dev,
                               int32_t F, int32_t T, const dmc_params* params,
                               void* frames_out_dev, dmc_window_stats* per_window);

/* ---- single steps of the path, for verification --------------------------
 * dmc_delta: delta = L V for each of F frames (Eq. 3-4): [F][n][3] ->
 *   [F][n][3] in the frames' dtype.
 * dmc_autocorrelation: R_c = A_c A_c^T (Eq. 7) of one T-frame window:
 *   frames [T][n][3] -> R_out_dev float64 [3][T][T]. */
dmc_status dmc_delta(dmc_ctx ctx, dmc_mesh mesh, const void* frames_dev, int32_t F,
                     int32_t precision, void* delta_out_dev);
dmc_status dmc_autocorrelation(dmc_ctx ctx, dmc_mesh mesh, const void* frames_dev,
                               int32_t T, int32_t precision, void* R_out_dev);

/* ---- orthogonal iterations on independent covariance blocks --------------
 * Algorithm 1's iterations and the Ritz step (as in dmc_encode_window) on nb
 * independent symmetric blocks R_dev float64 [nb][T][T], all concurrently:
 * U_out_dev float64 [nb][T][k] (k = params->k <= T), columns ordered by
 * eigenvalue, sign fixed.  params->init: DMC_INIT_RANDOM (q_start_dev
 * float64 [nb][T][k]), DMC_INIT_SKETCH (Omega float64 [T][k]),
 * DMC_INIT_EXACT, or DMC_INIT_LEARNED (registered network).  sweeps_host
 * [nb] and resid_host [nb] (optional; filling them synchronises) receive the
 * sweeps used and the final residual ||R Q - Q Q^T R Q||_F / ||R||_F. */
dmc_status dmc_oi_blocks(dmc_ctx ctx, const double* R_dev, int32_t nb, int32_t T,
                         const dmc_params* params, const void* q_start_dev,
                         double* U_out_dev, int32_t* sweeps_host, double* resid_host);

/* ---- learned start (not in the paper; the plain starts remain) ------------
 * A row-wise perceptron maps each row of the sketch features S (the columns
 * of R_c Omega, Omega [T][32], orthonormalised by Gram-Schmidt run twice, a
 * column keeping less than 1e-10 of its norm after the projections set to
 * zero, then scaled by sqrt(T)) to a row of the start block:
 * h1 = gelu(S W1 + b1) (32 -> 128), h2 = gelu(h1 W2 + b2) (128 -> 128),
 * Q = h2 W3 + b3 (128 -> k), gelu(x) = x Phi(x).  theta: float32
 * [dmc_mlp_param_count(k)] = W1 [32][128], b1 [128], W2 [128][128], b2 [128],
 * W3 [128][k], b3 [k], row-major.  Products take bfloat16 operands with
 * float32 accumulation (matrix cores); the backward pass uses the
 * bfloat16-rounded weights in float32.  All pointers are device memory;
 * every call is ordered on the context's stream.
 *
 * dmc_learned_start  registers (omega float64 [T][32], theta) for
 *                    DMC_INIT_LEARNED with this T and k; the buffers stay
 *                    owned by the caller and must outlive their use; NULL
 *                    pointers unregister.
 * dmc_mlp_sketch     S_out float32 [nb][T][32] from R float64 [nb][T][T].
 * dmc_mlp_forward    Q_out float32 [N][k] from S float32 [N][32]; cache
 *                    (optional, float32 [N][256]) keeps the pre-activations
 *                    for dmc_mlp_backward.
 * dmc_mlp_loss_grad  per block b of nb: loss_dev[b] (float64, optional) =
 *                    ||(I - U U^T) Q||^2 / ||Q||^2
 *                    + mu ||Q^T Q / (||Q||^2 / k) - I||^2 with Q float32 and
 *                    the orthonormal targets U float64, both [nb][T][k];
 *                    dQ_out float32 = gradient of the mean over blocks.
 * dmc_mlp_backward   grad_out float32 [count] = gradient of sum(dQ * Q) with
 *                    respect to theta (uses the context's scratch).
 * dmc_mlp_adam       one bias-corrected Adam step (step >= 1) on theta with
 *                    moments m, v (float32 [count], zero at step 1). */
int32_t dmc_mlp_param_count(int32_t k);
dmc_status dmc_learned_start(dmc_ctx ctx, int32_t T, int32_t k, const double* omega_dev,
                             const float* theta_dev);
dmc_status dmc_mlp_sketch(dmc_ctx ctx, const double* R_dev, int32_t nb, int32_t T,
                          const double* omega_dev, float* S_out_dev);
dmc_status dmc_mlp_forward(dmc_ctx ctx, const float* theta_dev, int32_t k, const float* S_dev,
                           int32_t N, float* Q_out_dev, float* cache_dev);
dmc_status dmc_mlp_loss_grad(dmc_ctx ctx, const float* Q_dev, const double* U_dev, int32_t nb,
                             int32_t T, int32_t k, double mu, float* dQ_out_dev,
                             double* loss_dev);
dmc_status dmc_mlp_backward(dmc_ctx ctx, const float* theta_dev, int32_t k, const float* S_dev,
                            int32_t N, const float* cache_dev, const float* dQ_dev,
                            float* grad_out_dev);
dmc_status dmc_mlp_adam(dmc_ctx ctx, float* theta_dev, const float* grad_dev, float* m_dev,
                        float* v_dev, int32_t count, int32_t step, double lr, double beta1,
                        double beta2, double eps);

/* ---- batched form: many independent sequences, one captured graph --------
 * dmc_batch_create plans nseq sequences: sequence i is frames_dev[i]
 * [F[i]][n_i][3] on meshes[i] (meshes of this context), windows of T[i],
 * params[i] (one precision for the whole batch; init DMC_INIT_PREV, _RANDOM,
 * _SKETCH or _EXACT with q_start_dev[i] as for dmc_compress_sequence),
 * records into codes_dev[i] (dmc_sequence_code_bytes bytes) and, when
 * frames_out_dev[i] is not NULL, the decoded frames.  Addresses are fixed at
 * creation: the first dmc_batch_run records the whole batch as a HIP graph
 * and later runs replay it.  In it the orthogonal iterations of every window
 * of every sequence run in one launch per class (T <= 32 or <= 64, k <= 16
 * or <= 32), the bandwidth-bound kernels per sequence, and each decode with
 * exactly params[i].cg_max_iters conjugate-gradient iterations and no host
 * synchronisation.  At creation a small autotuner times candidate vertex
 * splits of the covariance kernel on each sequence's own frames and keeps
 * the fastest.  Sequences are spread over four branches of the graph
 * (largest first onto the least loaded, by vertex-frames), each with its own
 * scratch: their kernels overlap on the GPU, those of one sequence run in
 * order.  The batch owns
 * its device scratch (allocated at creation); meshes and caller buffers must
 * outlive it.
 * dmc_batch_run: ordered on the context's stream, does not synchronise.
 * dmc_batch_stats: synchronises; fills per_window (one entry per window of
 * sequence seq) like dmc_compress_sequence (cg_iters = the fixed count,
 * cg_resid = largest relative residual) and returns DMC_ERR_NOT_CONVERGED if
 * some column of the sequence did not reach cg_tol.
 * dmc_batch_tuning: the autotuner's choices for sequence seq:
 * tuning[0] = covariance vertex blocks per window, tuning[1] = the graph
 * branch the sequence runs on (0-3). */
typedef struct dmc_batch_s* dmc_batch;
dmc_status dmc_batch_create(dmc_ctx ctx, int32_t nseq, const dmc_mesh* meshes,
                            const void* const* frames_dev, const int32_t* F, const int32_t* T,
                            const dmc_params* params, const void* const* q_start_dev,
                            void* const* codes_dev, void* const* frames_out_dev,
                            dmc_batch* out);
dmc_status dmc_batch_run(dmc_batch batch);
dmc_status dmc_batch_stats(dmc_batch batch, int32_t seq, dmc_window_stats* per_window);
dmc_status dmc_batch_tuning(dmc_batch batch, int32_t seq, int32_t tuning[2]);
void dmc_batch_destroy(dmc_batch batch);

/* ---- kernel timing (measurement support) ----------------------------------
 * dmc_profile_start selects one kernel family; from then on every launch of
 * it is bracketed by HIP events recorded on the stream it runs on.
 * dmc_profile_stop waits for those events and returns the number of launches
 * and their summed duration in milliseconds, then deselects.  Process-wide
 * state: use from one thread. */
enum {
  DMC_KERNEL_DELTA = 0, DMC_KERNEL_AUTOCORR, DMC_KERNEL_OI, DMC_KERNEL_PROJECT,
  DMC_KERNEL_QUANTISE, DMC_KERNEL_ANCHORS, DMC_KERNEL_BACK_PROJECT, DMC_KERNEL_RHS,
  DMC_KERNEL_CG_SPMM, DMC_KERNEL_CG_UPDATE, DMC_KERNEL_CHOL_FWD_GATHER,
  DMC_KERNEL_CHOL_FWD_SOLVE, DMC_KERNEL_CHOL_BWD_GATHER, DMC_KERNEL_CHOL_BWD_SOLVE,
  DMC_KERNEL_TO_FRAMES, DMC_KERNEL_COUNT
};
dmc_status dmc_profile_start(int32_t kernel);
dmc_status dmc_profile_stop(int32_t* launches, double* ms_total);

#ifdef __cplusplus
}
#endif
#endif /* DMC_H */
