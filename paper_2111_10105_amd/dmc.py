"""Thin ctypes binding of libdmc.so (include/dmc.h).

Argument marshalling only: every step of encode and decode runs in the HIP
library.  Device buffers are torch tensors on the GPU (torch is used for device
memory and streams); the library receives their raw pointers and the current
torch stream.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdmc.so")

DMC_OK = 0
NOALLOC_SCRATCH_BYTES = 64 << 20  # DMC_NOALLOC_SCRATCH_BYTES of include/dmc.h
STATUS = {0: "OK", 1: "INVALID_ARG", 2: "OUT_OF_MEMORY", 3: "DEVICE", 4: "NOT_CONVERGED",
          5: "SINGULAR", 6: "BUFFER_TOO_SMALL", 7: "UNSUPPORTED"}
FP64, FP32, BF16 = 0, 1, 2
LAP_UNIFORM, LAP_COMBINATORIAL = 0, 1
PRECOND_NONE, PRECOND_JACOBI, PRECOND_CHOLESKY = 0, 1, 2
INIT_PREV, INIT_RANDOM, INIT_SKETCH, INIT_EXACT, INIT_LEARNED = 0, 1, 2, 3, 4
DICT_PLAIN, DICT_ADAPTIVE = 0, 1

EXPORTS = ["dmc_create", "dmc_destroy", "dmc_set_stream", "dmc_last_error", "dmc_scratch_bytes",
           "dmc_workspace_bytes", "dmc_set_workspace",
           "dmc_mesh_create", "dmc_mesh_destroy", "dmc_mesh_nnz", "dmc_mesh_normal_nnz",
           "dmc_mesh_factor_info", "dmc_mesh_anchor_response", "dmc_host_normal_solve",
           "dmc_mesh_normal_solve",
           "dmc_window_code_bytes", "dmc_sequence_code_bytes", "dmc_encode_window",
           "dmc_encode_window_noalloc",
           "dmc_decode_window", "dmc_compress_sequence", "dmc_decode_sequence", "dmc_delta",
           "dmc_autocorrelation", "dmc_profile_start", "dmc_profile_stop", "dmc_oi_blocks",
           "dmc_mlp_param_count", "dmc_learned_start", "dmc_mlp_sketch", "dmc_mlp_forward",
           "dmc_mlp_loss_grad", "dmc_mlp_backward", "dmc_mlp_adam", "dmc_batch_create",
           "dmc_batch_run", "dmc_batch_stats", "dmc_batch_tuning", "dmc_batch_destroy"]

KERNELS = ["delta", "autocorr", "oi", "project", "quantise", "anchors", "back_project", "rhs",
           "cg_spmm", "cg_update", "chol_fwd_gather", "chol_fwd_solve", "chol_bwd_gather",
           "chol_bwd_solve", "to_frames"]


class DmcError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"dmc error {STATUS.get(status, status)}: {message}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("coef_bits", ctypes.c_int32),
                ("anchor_bits", ctypes.c_int32), ("dict_bits", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("oi_max_sweeps", ctypes.c_int32),
                ("oi_tol", ctypes.c_double), ("cg_max_iters", ctypes.c_int32),
                ("precond", ctypes.c_int32), ("cg_tol", ctypes.c_double),
                ("init", ctypes.c_int32), ("dict_mode", ctypes.c_int32),
                ("coef_step", ctypes.c_double)]


class WindowStats(ctypes.Structure):
    _fields_ = [("T", ctypes.c_int32), ("k", ctypes.c_int32),
                ("oi_sweeps", ctypes.c_int32 * 3), ("oi_resid", ctypes.c_double * 3),
                ("chol_shifts", ctypes.c_int32 * 3), ("cg_iters", ctypes.c_int32),
                ("cg_resid", ctypes.c_double), ("q", ctypes.c_double), ("q_a", ctypes.c_double),
                ("q_d", ctypes.c_double), ("q_s", ctypes.c_double),
                ("ms_encode", ctypes.c_float), ("ms_decode", ctypes.c_float)]

    def as_dict(self):
        return {"T": self.T, "k": self.k, "oi_sweeps": list(self.oi_sweeps),
                "oi_resid": list(self.oi_resid), "chol_shifts": list(self.chol_shifts),
                "cg_iters": self.cg_iters, "cg_resid": self.cg_resid, "q": self.q,
                "q_a": self.q_a, "q_d": self.q_d, "q_s": self.q_s,
                "ms_encode": self.ms_encode, "ms_decode": self.ms_decode}


def make_params(k, coef_bits=12, anchor_bits=16, dict_bits=16, precision=FP32,
                oi_max_sweeps=200, oi_tol=None, cg_max_iters=None, precond=PRECOND_CHOLESKY,
                cg_tol=None, init=INIT_PREV, dict_mode=0, coef_step=0.0) -> Params:
    if oi_tol is None:
        # the precision form's bfloat16 covariance fixes the trailing
        # eigen-directions only to its rounding: without a gap there the
        # residual stalls near 1e-8, so its default tolerance sits above that
        oi_tol = 1e-6 if precision == BF16 else 1e-12
    if cg_tol is None:
        cg_tol = 1e-12
    if cg_max_iters is None:
        cg_max_iters = 50 if precond == PRECOND_CHOLESKY else 20000
    return Params(k, coef_bits, anchor_bits, dict_bits, precision, oi_max_sweeps, float(oi_tol),
                  cg_max_iters, precond, float(cg_tol), init, dict_mode, float(coef_step))


_lib = None


def lib():
    """The loaded library; raises if it has not been built (there is no
    fallback implementation)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -c 'import __graft_entry__ as g; g.build()'`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, sz, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t, ctypes.c_double
    P = ctypes.POINTER(Params)
    S = ctypes.POINTER(WindowStats)
    sig = {
        "dmc_create": (i32, [i32, vp, ctypes.POINTER(vp)]),
        "dmc_destroy": (None, [vp]),
        "dmc_set_stream": (i32, [vp, vp]),
        "dmc_last_error": (ctypes.c_char_p, []),
        "dmc_scratch_bytes": (sz, [vp]),
        "dmc_workspace_bytes": (sz, [vp, i32, i32, P]),
        "dmc_set_workspace": (i32, [vp, vp, sz]),
        "dmc_mesh_create": (i32, [vp, i32, i32, vp, i32, vp, i32, ctypes.POINTER(vp)]),
        "dmc_mesh_destroy": (None, [vp]),
        "dmc_mesh_nnz": (i32, [vp]),
        "dmc_mesh_normal_nnz": (i32, [vp]),
        "dmc_mesh_factor_info": (None, [vp, ctypes.POINTER(dbl)]),
        "dmc_mesh_anchor_response": (i32, [vp, ctypes.POINTER(i32), ctypes.POINTER(dbl)]),
        "dmc_host_normal_solve": (i32, [i32, i32, vp, i32, vp, i32, i32, vp, vp,
                                        ctypes.POINTER(dbl)]),
        "dmc_window_code_bytes": (sz, [i32, i32, i32, P]),
        "dmc_sequence_code_bytes": (sz, [i32, i32, i32, i32, P]),
        "dmc_encode_window": (i32, [vp, vp, vp, i32, P, vp, vp, vp, vp, S]),
        "dmc_encode_window_noalloc": (i32, [vp, vp, vp, i32, P, vp, vp, vp, vp, S]),
        "dmc_decode_window": (i32, [vp, vp, vp, i32, P, vp, S]),
        "dmc_compress_sequence": (i32, [vp, vp, vp, i32, i32, P, vp, vp, sz, vp, S]),
        "dmc_decode_sequence": (i32, [vp, vp, vp, i32, i32, P, vp, S]),
        "dmc_delta": (i32, [vp, vp, vp, i32, i32, vp]),
        "dmc_mesh_normal_solve": (i32, [vp, vp, i32, vp, vp]),
        "dmc_autocorrelation": (i32, [vp, vp, vp, i32, i32, vp]),
        "dmc_profile_start": (i32, [i32]),
        "dmc_profile_stop": (i32, [ctypes.POINTER(i32), ctypes.POINTER(dbl)]),
        "dmc_oi_blocks": (i32, [vp, vp, i32, i32, P, vp, vp, vp, vp]),
        "dmc_mlp_param_count": (i32, [i32]),
        "dmc_learned_start": (i32, [vp, i32, i32, vp, vp]),
        "dmc_mlp_sketch": (i32, [vp, vp, i32, i32, vp, vp]),
        "dmc_mlp_forward": (i32, [vp, vp, i32, vp, i32, vp, vp]),
        "dmc_mlp_loss_grad": (i32, [vp, vp, vp, i32, i32, i32, dbl, vp, vp]),
        "dmc_mlp_backward": (i32, [vp, vp, i32, vp, i32, vp, vp, vp]),
        "dmc_mlp_adam": (i32, [vp, vp, vp, vp, vp, i32, i32, dbl, dbl, dbl, dbl]),
        "dmc_batch_create": (i32, [vp, i32, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                   ctypes.POINTER(i32), ctypes.POINTER(i32), P, ctypes.POINTER(vp),
                                   ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp)]),
        "dmc_batch_run": (i32, [vp]),
        "dmc_batch_stats": (i32, [vp, i32, S]),
        "dmc_batch_tuning": (i32, [vp, i32, ctypes.POINTER(i32)]),
        "dmc_batch_destroy": (None, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(status: int, allow=()):
    if status != DMC_OK and status not in allow:
        raise DmcError(status, lib().dmc_last_error().decode())
    return status


def _check_start(q_start, frames, T: int, params: "Params", nw: int = 0):
    """Shape, dtype and device of a start block (the library reads it as raw
    memory): [3][T][k] (DMC_INIT_PREV; DMC_INIT_RANDOM for one window),
    [nw][3][T][k] (DMC_INIT_RANDOM over nw full windows), Omega [T][k]
    (DMC_INIT_SKETCH); k = min(params.k, T)."""
    if q_start is None or params.init == INIT_EXACT:
        return
    k = min(params.k, T)
    if params.init == INIT_SKETCH:
        want = (T, k)
    elif params.init == INIT_RANDOM and nw:
        want = (nw, 3, T, k)
    else:
        want = (3, T, k)
    if tuple(q_start.shape) != want:
        raise ValueError(f"q_start must have shape {want}, got {tuple(q_start.shape)}")
    if q_start.dtype != frames.dtype or q_start.device != frames.device:
        raise ValueError("q_start must match the frames' dtype and device")
    if not q_start.is_contiguous():
        raise ValueError("q_start must be contiguous")


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _real(precision):
    import torch
    return torch.float64 if precision == FP64 else torch.float32


class Context:
    def __init__(self, device: int = 0):
        import torch
        torch.cuda.set_device(device)
        h = ctypes.c_void_p()
        _check(lib().dmc_create(device, _stream(), ctypes.byref(h)))
        self.h = h
        self.device = device

    def sync_stream(self):
        _check(lib().dmc_set_stream(self.h, _stream()))

    @property
    def scratch_bytes(self) -> int:
        return lib().dmc_scratch_bytes(self.h)

    def set_workspace(self, buf):
        """Use a caller-owned device buffer (a uint8 CUDA tensor, or None to
        return to library-allocated scratch) as the context's scratch; the
        context keeps a reference to the tensor."""
        self.sync_stream()
        if buf is None:
            _check(lib().dmc_set_workspace(self.h, None, 0))
        else:
            _check(lib().dmc_set_workspace(self.h, _ptr(buf), buf.numel() * buf.element_size()))
        self._workspace = buf

    def close(self):
        if self.h:
            lib().dmc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Mesh:
    def __init__(self, ctx: Context, n: int, tris, anchors, laplacian: int = LAP_UNIFORM):
        tris = np.ascontiguousarray(tris, dtype=np.int32)
        anchors = np.ascontiguousarray(anchors, dtype=np.int32)
        h = ctypes.c_void_p()
        _check(lib().dmc_mesh_create(ctx.h, int(n), int(tris.shape[0]),
                                     tris.ctypes.data_as(ctypes.c_void_p), int(anchors.size),
                                     anchors.ctypes.data_as(ctypes.c_void_p), int(laplacian),
                                     ctypes.byref(h)))
        self.h, self.ctx, self.n, self.nc = h, ctx, int(n), int(anchors.size)
        self.anchors = anchors

    @property
    def nnz(self):
        return lib().dmc_mesh_nnz(self.h)

    @property
    def normal_nnz(self):
        return lib().dmc_mesh_normal_nnz(self.h)

    def factor_info(self) -> dict:
        a = (ctypes.c_double * len(FACTOR_INFO_KEYS))()
        lib().dmc_mesh_factor_info(self.h, a)
        return dict(zip(FACTOR_INFO_KEYS, list(a)))

    def anchor_response(self):
        """(built, CG iterations, largest relative residual) of the mesh's
        anchor response (see dmc_mesh_anchor_response): with it the decoder
        solves 3k columns per window instead of 3T."""
        it = ctypes.c_int32(0)
        res = ctypes.c_double(0.0)
        built = lib().dmc_mesh_anchor_response(self.h, ctypes.byref(it), ctypes.byref(res))
        return bool(built), int(it.value), float(res.value)


FACTOR_INFO_KEYS = ("stored", "nnz_exact", "supernodes", "levels", "flops", "seconds",
                    "solve_entries", "update_rows", "leaf_rows")


def host_normal_solve(n, tris, anchors, B, laplacian: int = LAP_UNIFORM):
    """Solve (L^T L + I_N^T I_N) X = B on the host with the library's own
    ordering, factorisation and blocked triangular solves (no GPU)."""
    tris = np.ascontiguousarray(tris, dtype=np.int32)
    anchors = np.ascontiguousarray(anchors, dtype=np.int32)
    B = np.ascontiguousarray(B, dtype=np.float64)
    if B.ndim == 1:
        B = B[:, None]
    X = np.empty_like(B)
    info = (ctypes.c_double * len(FACTOR_INFO_KEYS))()
    _check(lib().dmc_host_normal_solve(int(n), int(tris.shape[0]), tris.ctypes.data_as(ctypes.c_void_p),
                                       int(anchors.size), anchors.ctypes.data_as(ctypes.c_void_p),
                                       int(laplacian), int(B.shape[1]),
                                       B.ctypes.data_as(ctypes.c_void_p),
                                       X.ctypes.data_as(ctypes.c_void_p), info))
    return X, dict(zip(FACTOR_INFO_KEYS, list(info)))


def workspace_bytes(mesh: "Mesh", F: int, T: int, params: Params) -> int:
    return lib().dmc_workspace_bytes(mesh.h, int(F), int(T), ctypes.byref(params))


def window_code_bytes(n, T, nc, params: Params) -> int:
    return lib().dmc_window_code_bytes(n, T, nc, ctypes.byref(params))


def sequence_code_bytes(n, F, T, nc, params: Params) -> int:
    return lib().dmc_sequence_code_bytes(n, F, T, nc, ctypes.byref(params))


def encode_window(ctx: Context, mesh: Mesh, frames, params: Params, q_start=None,
                  want_u: bool = True, want_coef: bool = False, stats: bool = True):
    """frames: CUDA tensor [T][n][3].  Returns a dict with the record (uint8
    tensor), U_k [3][T][k], coefficients [3][k][n] (if asked) and stats."""
    import torch
    T = frames.shape[0]
    dev = frames.device
    _check_start(q_start, frames, T, params)
    ctx.sync_stream()
    code = torch.empty(window_code_bytes(mesh.n, T, mesh.nc, params), dtype=torch.uint8, device=dev)
    k = min(params.k, T)
    u = torch.empty((3, T, k), dtype=frames.dtype, device=dev) if want_u else None
    coef = torch.empty((3, k, mesh.n), dtype=frames.dtype, device=dev) if want_coef else None
    st = WindowStats()
    status = lib().dmc_encode_window(ctx.h, mesh.h, _ptr(frames), T, ctypes.byref(params),
                                     _ptr(q_start), _ptr(code), _ptr(u), _ptr(coef),
                                     ctypes.byref(st) if stats else None)
    _check(status, allow=(4,))
    return {"code": code, "u": u, "coef": coef, "stats": st.as_dict() if stats else None,
            "status": status}


def decode_window(ctx: Context, mesh: Mesh, code, T: int, params: Params, dtype=None):
    import torch
    ctx.sync_stream()
    out = torch.empty((T, mesh.n, 3), dtype=dtype or _real(params.precision), device=code.device)
    st = WindowStats()
    status = lib().dmc_decode_window(ctx.h, mesh.h, _ptr(code), T, ctypes.byref(params),
                                     _ptr(out), ctypes.byref(st))
    _check(status, allow=(4,))
    return out, st.as_dict(), status


def compress_sequence(ctx: Context, mesh: Mesh, frames, T: int, params: Params, q_start=None,
                      decode: bool = True, stats: bool = True, codes=None, out=None):
    """Encode (and decode) a whole sequence [F][n][3].  Returns (codes, frames
    or None, per-window stats list, status)."""
    import torch
    F = frames.shape[0]
    _check_start(q_start, frames, T, params, nw=F // T)
    ctx.sync_stream()
    nbytes = sequence_code_bytes(mesh.n, F, T, mesh.nc, params)
    if codes is None:
        codes = torch.empty(nbytes, dtype=torch.uint8, device=frames.device)
    if decode and out is None:
        out = torch.empty_like(frames)
    nw = (F + T - 1) // T
    sts = (WindowStats * nw)() if stats else None
    status = lib().dmc_compress_sequence(ctx.h, mesh.h, _ptr(frames), F, T, ctypes.byref(params),
                                         _ptr(q_start), _ptr(codes), nbytes,
                                         _ptr(out) if decode else None, sts)
    _check(status, allow=(4,))
    return codes, (out if decode else None), ([s.as_dict() for s in sts] if stats else None), status


def decode_sequence(ctx: Context, mesh: Mesh, codes, F: int, T: int, params: Params, out=None):
    import torch
    ctx.sync_stream()
    if out is None:
        out = torch.empty((F, mesh.n, 3), dtype=_real(params.precision), device=codes.device)
    nw = (F + T - 1) // T
    sts = (WindowStats * nw)()
    status = lib().dmc_decode_sequence(ctx.h, mesh.h, _ptr(codes), F, T, ctypes.byref(params),
                                       _ptr(out), sts)
    _check(status, allow=(4,))
    return out, [s.as_dict() for s in sts], status


def normal_solve(ctx: Context, mesh: Mesh, B):
    """X with (L^T L + I_N^T I_N) X = B by the mesh's device Cholesky factor
    (dmc_mesh_normal_solve); B float64 [n][ncols] on the device."""
    import torch
    assert B.dtype == torch.float64 and B.dim() == 2 and B.shape[0] == mesh.n
    B = B.contiguous()
    ctx.sync_stream()
    X = torch.empty_like(B)
    _check(lib().dmc_mesh_normal_solve(ctx.h, mesh.h, int(B.shape[1]), _ptr(B), _ptr(X)))
    return X


def delta(ctx: Context, mesh: Mesh, frames, precision: int):
    import torch
    ctx.sync_stream()
    out = torch.empty_like(frames)
    _check(lib().dmc_delta(ctx.h, mesh.h, _ptr(frames), frames.shape[0], precision, _ptr(out)))
    return out


def autocorrelation(ctx: Context, mesh: Mesh, frames, precision: int):
    import torch
    ctx.sync_stream()
    T = frames.shape[0]
    R = torch.empty((3, T, T), dtype=torch.float64, device=frames.device)
    _check(lib().dmc_autocorrelation(ctx.h, mesh.h, _ptr(frames), T, precision, _ptr(R)))
    return R


def profile_start(kernel: str):
    """Time every launch of one kernel family with HIP events from now on."""
    _check(lib().dmc_profile_start(KERNELS.index(kernel)))


def profile_stop():
    """(launches, total milliseconds) of the selected kernel family."""
    n = ctypes.c_int32()
    ms = ctypes.c_double()
    _check(lib().dmc_profile_stop(ctypes.byref(n), ctypes.byref(ms)))
    return n.value, ms.value


# ---- record parsing (host side, for inspection and tests) --------------------

def _align(x, a=256):
    return (x + a - 1) // a * a


def _seg_words(count, bits, real):
    w = (count * bits + 31) // 32 if bits else (count * real + 3) // 4
    return w + (w & 1)


def _unpack(words, count, bits):
    """Codes of a packed segment (LSB first within 32-bit words)."""
    if bits == 0 or count == 0:
        return np.zeros(count, dtype=np.uint32)
    w = np.asarray(words, dtype=np.uint64)
    pos = np.arange(count, dtype=np.uint64) * np.uint64(bits)
    wi = (pos >> np.uint64(5)).astype(np.int64)
    sh = pos & np.uint64(31)
    hi = np.where(wi + 1 < w.size, w[np.minimum(wi + 1, w.size - 1)], 0).astype(np.uint64)
    both = w[wi] | (hi << np.uint64(32))
    return ((both >> sh) & np.uint64((1 << bits) - 1)).astype(np.uint32)


HEADER_WORDS = 32
SEG_DTYPE = np.dtype([("lo", "<f4"), ("hi", "<f4"), ("bits_mode", "<u4"), ("word_off", "<u4")])


@dataclass
class RecordView:
    header: np.ndarray          # int32 [32]
    dict_table: np.ndarray      # [3][k] (lo, hi, bits_mode, word_off)
    dict_codes: np.ndarray      # [3][T][k] codes (uint32) or raw values
    ranges: np.ndarray | None   # [3][k][2] float32 (None for raw rows)
    row_bits: np.ndarray        # [3][k]
    codes: np.ndarray           # [3][k][n] codes (uint32) or raw values
    anchor_range: np.ndarray | None  # [3][2] float32
    anchor_codes: np.ndarray    # [3][T][nc] codes (uint32) or raw values
    used_bytes: int
    var_words: np.ndarray       # the variable part's 32-bit words (dictionary, then rows)
    anchor_words: list          # [3] words of the anchor segments

    @property
    def dict_bits(self):
        return self.dict_table["bits_mode"] & 0xFF

    @property
    def dict_modes(self):
        return (self.dict_table["bits_mode"] >> 8) & 0xFF


def parse_record(buf: np.ndarray, n: int, T: int, nc: int, params: Params) -> RecordView:
    """Split one record (bytes copied to the host) into its header, tables and
    unpacked codes; mirrors the layout documented in dmc.h."""
    buf = np.asarray(buf, dtype=np.uint8)
    k = min(params.k, T)
    real = np.float64 if params.precision == FP64 else np.float32
    rs = np.dtype(real).itemsize
    hdr = buf[:128].view(np.int32).copy()
    off_dtab = 128
    off_rtab = off_dtab + 3 * k * 16
    off_arange = off_rtab + 3 * k * 16
    off_anchors = _align(off_arange + 24)
    aseg = 4 * _seg_words(T * nc, params.anchor_bits, rs)
    off_var = _align(off_anchors + 3 * aseg)
    dtab = buf[off_dtab:off_rtab].view(SEG_DTYPE).reshape(3, k).copy()
    rtab = buf[off_rtab:off_arange].view(SEG_DTYPE).reshape(3, k).copy()
    arng = buf[off_arange:off_arange + 24].view(np.float32).reshape(3, 2).copy()
    used = int(np.uint32(hdr[11])) | (int(np.uint32(hdr[12])) << 32)
    var = buf[off_var:used].view(np.uint32)
    dict_codes = np.zeros((3, T, k), dtype=real if params.dict_bits == 0 else np.uint32)
    for c in range(3):
        for j in range(k):
            e = dtab[c, j]
            b = int(e["bits_mode"]) & 0xFF
            o = int(e["word_off"])
            nwd = _seg_words(T, b if params.dict_bits else 0, rs)
            words = var[o:o + nwd]
            if params.dict_bits == 0:
                dict_codes[c, :, j] = words.view(real)[:T]
            else:
                dict_codes[c, :, j] = _unpack(words, T, b)
    codes = np.zeros((3, k, n), dtype=real if params.coef_bits == 0 else np.uint32)
    row_bits = (rtab["bits_mode"] & 0xFF).astype(np.int64)
    for c in range(3):
        for r in range(k):
            b = int(row_bits[c, r])
            o = int(rtab[c, r]["word_off"])
            nwd = _seg_words(n, b if params.coef_bits else 0, rs)
            words = var[o:o + nwd]
            codes[c, r] = words.view(real)[:n] if params.coef_bits == 0 else _unpack(words, n, b)
    ranges = np.stack([rtab["lo"], rtab["hi"]], axis=-1).astype(np.float32)
    anc = np.zeros((3, T, nc), dtype=real if params.anchor_bits == 0 else np.uint32)
    aw = []
    for c in range(3):
        words = buf[off_anchors + c * aseg:off_anchors + (c + 1) * aseg].view(np.uint32)
        aw.append(words)
        if params.anchor_bits == 0:
            anc[c] = words.view(real)[:T * nc].reshape(T, nc)
        else:
            anc[c] = _unpack(words, T * nc, params.anchor_bits).reshape(T, nc)
    return RecordView(hdr, dtab, dict_codes, ranges if params.coef_bits > 0 else None, row_bits,
                      codes, arng if params.anchor_bits > 0 else None, anc, used, var, aw)


# ---- orthogonal iterations on independent blocks, learned start ------------

def _need(t, dtype, shape, name):
    import torch
    if t.dtype != dtype or tuple(t.shape) != tuple(shape) or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous CUDA {dtype} tensor of shape {tuple(shape)}, "
                         f"got {t.dtype} {tuple(t.shape)}")


def oi_blocks(ctx: Context, R, params: Params, q_start=None):
    """Orthogonal iterations + Ritz step on independent blocks R float64
    [nb][T][T]; returns (U float64 [nb][T][k], sweeps, residuals) as
    (tensor, numpy int32, numpy float64)."""
    import torch
    nb, T = R.shape[0], R.shape[1]
    _need(R, torch.float64, (nb, T, T), "R")
    k = params.k
    if q_start is not None:
        want = (T, k) if params.init == INIT_SKETCH else (nb, T, k)
        _need(q_start, torch.float64, want, "q_start")
    ctx.sync_stream()
    U = torch.empty((nb, T, k), dtype=torch.float64, device=R.device)
    sweeps = np.zeros(nb, dtype=np.int32)
    resid = np.zeros(nb, dtype=np.float64)
    _check(lib().dmc_oi_blocks(ctx.h, _ptr(R), nb, T, ctypes.byref(params), _ptr(q_start), _ptr(U),
                               sweeps.ctypes.data_as(ctypes.c_void_p),
                               resid.ctypes.data_as(ctypes.c_void_p)))
    return U, sweeps, resid


def mlp_param_count(k: int) -> int:
    return int(lib().dmc_mlp_param_count(int(k)))


def learned_start(ctx: Context, T: int, k: int, omega, theta):
    """Register (omega float64 [T][32], theta float32) for INIT_LEARNED; the
    context keeps references to both tensors.  None unregisters."""
    import torch
    if omega is None or theta is None:
        _check(lib().dmc_learned_start(ctx.h, 0, 0, None, None))
        ctx._learned = None
        return
    _need(omega, torch.float64, (T, 32), "omega")
    _need(theta, torch.float32, (mlp_param_count(k),), "theta")
    _check(lib().dmc_learned_start(ctx.h, int(T), int(k), _ptr(omega), _ptr(theta)))
    ctx._learned = (omega, theta)


def mlp_sketch(ctx: Context, R, omega):
    import torch
    nb, T = R.shape[0], R.shape[1]
    _need(R, torch.float64, (nb, T, T), "R")
    _need(omega, torch.float64, (T, 32), "omega")
    ctx.sync_stream()
    S = torch.empty((nb, T, 32), dtype=torch.float32, device=R.device)
    _check(lib().dmc_mlp_sketch(ctx.h, _ptr(R), nb, T, _ptr(omega), _ptr(S)))
    return S


def mlp_forward(ctx: Context, theta, k: int, S, cache: bool = False):
    """Rows of S float32 [N][32] (any leading shape) -> Q float32 [N][k];
    with cache=True also the pre-activations [N][256] for mlp_backward."""
    import torch
    N = S.numel() // 32
    _need(theta, torch.float32, (mlp_param_count(k),), "theta")
    if S.dtype != torch.float32 or not S.is_contiguous() or S.shape[-1] != 32:
        raise ValueError("S must be contiguous float32 with 32 columns")
    ctx.sync_stream()
    Q = torch.empty((N, k), dtype=torch.float32, device=S.device)
    C = torch.empty((N, 256), dtype=torch.float32, device=S.device) if cache else None
    _check(lib().dmc_mlp_forward(ctx.h, _ptr(theta), int(k), _ptr(S), N, _ptr(Q), _ptr(C)))
    return (Q, C) if cache else Q


def mlp_loss_grad(ctx: Context, Q, U, mu: float = 0.1):
    """Q float32 and U float64, both [nb][T][k] -> (dQ float32 [nb][T][k],
    per-block losses float64 [nb])."""
    import torch
    nb, T, k = U.shape
    _need(U, torch.float64, (nb, T, k), "U")
    _need(Q, torch.float32, (nb, T, k), "Q")
    ctx.sync_stream()
    dQ = torch.empty_like(Q)
    loss = torch.empty(nb, dtype=torch.float64, device=Q.device)
    _check(lib().dmc_mlp_loss_grad(ctx.h, _ptr(Q), _ptr(U), nb, T, k, float(mu), _ptr(dQ), _ptr(loss)))
    return dQ, loss


def mlp_backward(ctx: Context, theta, k: int, S, cache, dQ):
    import torch
    N = S.numel() // 32
    _need(cache, torch.float32, (N, 256), "cache")
    if dQ.numel() != N * k or dQ.dtype != torch.float32 or not dQ.is_contiguous():
        raise ValueError("dQ must be contiguous float32 with N x k entries")
    ctx.sync_stream()
    g = torch.empty_like(theta)
    _check(lib().dmc_mlp_backward(ctx.h, _ptr(theta), int(k), _ptr(S), N, _ptr(cache), _ptr(dQ),
                                  _ptr(g)))
    return g


def mlp_adam(ctx: Context, theta, grad, m, v, step: int, lr: float, beta1: float = 0.9,
             beta2: float = 0.999, eps: float = 1e-8):
    """One Adam step in place on theta, m, v (float32 tensors of one size)."""
    ctx.sync_stream()
    _check(lib().dmc_mlp_adam(ctx.h, _ptr(theta), _ptr(grad), _ptr(m), _ptr(v), theta.numel(),
                              int(step), float(lr), float(beta1), float(beta2), float(eps)))


# ---- batched form ------------------------------------------------------------

class Batch:
    """Many independent sequences encoded and decoded by one replayed HIP
    graph.  frames: list of CUDA tensors [F_i][n_i][3] (one dtype), meshes:
    list of Mesh, Ts: window lengths, params: list of Params (one precision),
    q_starts: optional list of start blocks (as for compress_sequence).  The
    batch allocates each sequence's record buffer and (with decode=True) its
    output frames; their addresses stay fixed for the life of the batch."""

    def __init__(self, ctx: Context, meshes, frames, Ts, params, q_starts=None, decode=True):
        import torch
        nseq = len(frames)
        if not (len(meshes) == len(Ts) == len(params) == nseq) or nseq < 1:
            raise ValueError("meshes, frames, Ts and params must have one entry per sequence")
        ctx.sync_stream()
        self.ctx = ctx
        self.frames = frames
        self.meshes = meshes
        self.Ts = [int(t) for t in Ts]
        self.params = list(params)
        self.q_starts = list(q_starts) if q_starts is not None else [None] * nseq
        for f, T, p, q in zip(frames, self.Ts, self.params, self.q_starts):
            if not f.is_cuda or not f.is_contiguous():
                raise ValueError("frames must be contiguous CUDA tensors")
            _check_start(q, f, T, p, nw=f.shape[0] // T)
        self.codes = [torch.empty(sequence_code_bytes(m.n, f.shape[0], T, m.nc, p), dtype=torch.uint8,
                                  device=f.device)
                      for m, f, T, p in zip(meshes, frames, self.Ts, self.params)]
        self.out = [torch.empty_like(f) for f in frames] if decode else None
        vpa = ctypes.c_void_p * nseq
        P = (Params * nseq)(*self.params)
        h = ctypes.c_void_p()
        _check(lib().dmc_batch_create(
            ctx.h, nseq, vpa(*[m.h for m in meshes]), vpa(*[f.data_ptr() for f in frames]),
            (ctypes.c_int32 * nseq)(*[f.shape[0] for f in frames]), (ctypes.c_int32 * nseq)(*self.Ts),
            P, vpa(*[q.data_ptr() if q is not None else None for q in self.q_starts]),
            vpa(*[c.data_ptr() for c in self.codes]),
            vpa(*[o.data_ptr() for o in self.out]) if decode else None, ctypes.byref(h)))
        self.h = h

    def run(self):
        self.ctx.sync_stream()
        _check(lib().dmc_batch_run(self.h))

    def stats(self, i: int):
        nw = (self.frames[i].shape[0] + self.Ts[i] - 1) // self.Ts[i]
        sts = (WindowStats * nw)()
        status = lib().dmc_batch_stats(self.h, int(i), sts)
        _check(status, allow=(4,))
        return [s.as_dict() for s in sts], status

    def tuning(self, i: int):
        t = (ctypes.c_int32 * 2)()
        _check(lib().dmc_batch_tuning(self.h, int(i), t))
        return {"autocorr_blocks": t[0], "branch": t[1]}

    def close(self):
        if self.h:
            lib().dmc_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

