"""Truncated SVD by the power method on MI355X (gfx950): Python binding.

A thin ctypes layer over libtsvd.so (declared in include/tsvd.h).  Functions
keep the C names and only marshal arguments: torch tensors supply device
memory and the current HIP stream; every step of the computation runs in the
library's HIP kernels.  There is no fallback: if the library is not built, or
no GPU is present, the calls raise.

Layouts follow the C ABI: A is row-major; U (m x k) and V (n x k) come back as
column-major matrices, i.e. torch views ``t.T`` of contiguous (k, m) / (k, n)
tensors, so column j is contiguous; S is float64.
"""

from __future__ import annotations

import ctypes
import os

__all__ = [
    "TsvdError",
    "Context",
    "load_library",
    "library_path",
    "STATUS",
    "tsvd_gram_dense",
    "tsvd_power_gram",
    "tsvd_finish_dense",
    "tsvd_dense",
    "tsvd_dense_batched",
    "Server",
    "set_tuning",
    "get_tuning",
    "gram_class",
    "GRAM_CLASSES",
    "Csr",
    "tsvd_csr_create",
    "tsvd_csr_create_pinned",
    "tsvd_csr_get_csc",
    "tsvd_spmv",
    "tsvd_sparse",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_NAME = "libtsvd.so"

STATUS = {
    0: "TSVD_OK",
    1: "TSVD_ERR_INVALID_ARG",
    2: "TSVD_ERR_OUT_OF_MEMORY",
    3: "TSVD_ERR_NOT_CONVERGED",
    4: "TSVD_ERR_NONFINITE",
    5: "TSVD_ERR_HIP",
    6: "TSVD_ERR_REJECTED",
    7: "TSVD_ERR_UNSUPPORTED",
    8: "TSVD_ERR_INTERNAL",
}
OK, INVALID_ARG, OUT_OF_MEMORY, NOT_CONVERGED, NONFINITE, HIP, REJECTED, UNSUPPORTED, INTERNAL = range(9)

F32, F64 = 0, 1
LOC_DEVICE, LOC_PINNED_HOST = 0, 1
GRAM = {"auto": 0, "fp32": 1, "bf16x3": 2, "fp64": 3}
METHOD = {"auto": 0, "gram": 1, "implicit": 2}
SIDE = {"right": 0, "left": 1}


class TsvdError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        self.name = STATUS.get(status, str(status))
        super().__init__(f"{self.name}: {message}")


class TsvdOpts(ctypes.Structure):
    _fields_ = [
        ("k", ctypes.c_int32),
        ("eps", ctypes.c_double),
        ("max_iter", ctypes.c_int32),
        ("fixed_iters", ctypes.POINTER(ctypes.c_int32)),
        ("v0", ctypes.c_void_p),
        ("gram", ctypes.c_int32),
        ("rows_per_block", ctypes.c_int64),
        ("hbm_budget", ctypes.c_int64),
        ("branch", ctypes.c_int32),
        ("queue_depth", ctypes.c_int32),
        ("method", ctypes.c_int32),
        ("factor_loc", ctypes.c_int32),
        ("factor_batches", ctypes.c_int32),
    ]


GRAM_CLASSES = 8  # Gram-dimension classes of the batched Gram's unit shapes


def gram_class(d: int) -> int:
    """Class of a Gram dimension: 0 for d <= 128, c for 2^(6+c) < d <= 2^(7+c),
    the last class for anything larger."""
    c = 0
    while c < GRAM_CLASSES - 1 and d > (128 << c):
        c += 1
    return c


class TsvdTuning(ctypes.Structure):
    _fields_ = [
        ("gram_tile", ctypes.c_int32),
        ("gram_chunks", ctypes.c_int32),
        ("power_blocks", ctypes.c_int32),
        ("team_kib", ctypes.c_int32),
        ("group_kchunk", ctypes.c_int32),
        ("sparse_row_bits", ctypes.c_int32),
        ("sparse_col_bits", ctypes.c_int32),
        ("power_path", ctypes.c_int32),
        ("group_tile", ctypes.c_int32 * GRAM_CLASSES),
        ("group_kchunk_cls", ctypes.c_int32 * GRAM_CLASSES),
    ]


class TsvdProblem(ctypes.Structure):
    _fields_ = [
        ("A", ctypes.c_void_p),
        ("dtype", ctypes.c_int32),
        ("m", ctypes.c_int64),
        ("n", ctypes.c_int64),
        ("lda", ctypes.c_int64),
        ("opts", TsvdOpts),
        ("U", ctypes.c_void_p),
        ("ldu", ctypes.c_int64),
        ("S", ctypes.c_void_p),
        ("V", ctypes.c_void_p),
        ("ldv", ctypes.c_int64),
    ]


class TsvdServerConfig(ctypes.Structure):
    _fields_ = [
        ("hbm_budget", ctypes.c_int64),
        ("max_slots", ctypes.c_int32),
        ("max_batch", ctypes.c_int32),
        ("lanes", ctypes.c_int32),
    ]


class TsvdServerStats(ctypes.Structure):
    _fields_ = [
        ("submitted", ctypes.c_int64),
        ("completed", ctypes.c_int64),
        ("failed", ctypes.c_int64),
        ("rejected", ctypes.c_int64),
        ("batches", ctypes.c_int64),
        ("mean_batch", ctypes.c_double),
        ("p50_ms", ctypes.c_double),
        ("p99_ms", ctypes.c_double),
        ("mean_ms", ctypes.c_double),
        ("max_ms", ctypes.c_double),
        ("peak_bytes", ctypes.c_int64),
        ("in_flight", ctypes.c_int64),
        ("waiting", ctypes.c_int64),
        ("lanes_busy_max", ctypes.c_int64),
        ("overlapped", ctypes.c_int64),
    ]


class TsvdInfo(ctypes.Structure):
    _fields_ = [
        ("k_done", ctypes.c_int32),
        ("rank_deficient", ctypes.c_int32),
        ("converged", ctypes.c_int32),
        ("branch_right", ctypes.c_int32),
        ("iters", ctypes.POINTER(ctypes.c_int32)),
        ("lambda_", ctypes.POINTER(ctypes.c_double)),
        ("t_gram_ms", ctypes.c_double),
        ("t_eig_ms", ctypes.c_double),
        ("t_final_ms", ctypes.c_double),
        ("t_total_ms", ctypes.c_double),
        ("workspace_bytes", ctypes.c_int64),
        ("h2d_bytes", ctypes.c_int64),
        ("latency_ms", ctypes.c_double),
        ("t_stream_copy_ms", ctypes.c_double),
        ("t_stream_compute_ms", ctypes.c_double),
        ("t_stream_overlap_ms", ctypes.c_double),
    ]


_lib = None


def library_path() -> str:
    return os.path.join(_HERE, _LIB_NAME)


def load_library():
    """Load libtsvd.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    path = library_path()
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2208_08410_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.tsvd_ctx_create.argtypes = [ctypes.c_int, ctypes.POINTER(vp)]
    lib.tsvd_ctx_create.restype = ctypes.c_int
    lib.tsvd_ctx_destroy.argtypes = [vp]
    lib.tsvd_ctx_destroy.restype = None
    lib.tsvd_status_string.argtypes = [ctypes.c_int]
    lib.tsvd_status_string.restype = ctypes.c_char_p
    lib.tsvd_last_error.argtypes = [vp]
    lib.tsvd_last_error.restype = ctypes.c_char_p
    lib.tsvd_opts_default.argtypes = [ctypes.POINTER(TsvdOpts)]
    lib.tsvd_opts_default.restype = None
    lib.tsvd_gram_dense.argtypes = [vp, vp, i32, i64, i64, i64, i32, i32, i64, vp, i64, i32, vp]
    lib.tsvd_gram_dense.restype = ctypes.c_int
    lib.tsvd_power_gram.argtypes = [vp, vp, i32, i64, i64, ctypes.POINTER(TsvdOpts), vp, i64,
                                    ctypes.POINTER(TsvdInfo), vp]
    lib.tsvd_power_gram.restype = ctypes.c_int
    lib.tsvd_finish_dense.argtypes = [vp, vp, i32, i64, i64, i64, i32, vp, i64, i32, vp, i64, vp, vp]
    lib.tsvd_finish_dense.restype = ctypes.c_int
    lib.tsvd_dense.argtypes = [vp, vp, i32, i32, i64, i64, i64, ctypes.POINTER(TsvdOpts), vp, i64, vp, vp, i64,
                               ctypes.POINTER(TsvdInfo), vp]
    lib.tsvd_dense.restype = ctypes.c_int
    lib.tsvd_dense_batched.argtypes = [vp, i32, ctypes.POINTER(TsvdProblem), i64, ctypes.POINTER(TsvdInfo),
                                       ctypes.POINTER(ctypes.c_int32), vp]
    lib.tsvd_dense_batched.restype = ctypes.c_int
    lib.tsvd_server_create.argtypes = [vp, ctypes.POINTER(TsvdServerConfig), ctypes.POINTER(vp)]
    lib.tsvd_server_create.restype = ctypes.c_int
    lib.tsvd_server_submit.argtypes = [vp, ctypes.POINTER(TsvdProblem), i32, ctypes.POINTER(ctypes.c_uint64)]
    lib.tsvd_server_submit.restype = ctypes.c_int
    lib.tsvd_server_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(i32), ctypes.POINTER(TsvdInfo),
                                     ctypes.POINTER(i32)]
    lib.tsvd_server_poll.restype = ctypes.c_int
    lib.tsvd_server_wait.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(TsvdInfo)]
    lib.tsvd_server_wait.restype = ctypes.c_int
    lib.tsvd_server_get_stats.argtypes = [vp, ctypes.POINTER(TsvdServerStats)]
    lib.tsvd_server_get_stats.restype = ctypes.c_int
    lib.tsvd_server_last_error.argtypes = [vp]
    lib.tsvd_server_last_error.restype = ctypes.c_char_p
    lib.tsvd_server_destroy.argtypes = [vp]
    lib.tsvd_server_destroy.restype = None
    lib.tsvd_ctx_set_tuning.argtypes = [vp, ctypes.POINTER(TsvdTuning)]
    lib.tsvd_ctx_set_tuning.restype = ctypes.c_int
    lib.tsvd_ctx_get_tuning.argtypes = [vp, ctypes.POINTER(TsvdTuning)]
    lib.tsvd_ctx_get_tuning.restype = ctypes.c_int
    lib.tsvd_csr_create.argtypes = [vp, i64, i64, i64, vp, vp, vp, ctypes.POINTER(vp), vp]
    lib.tsvd_csr_create.restype = ctypes.c_int
    lib.tsvd_csr_create_pinned.argtypes = [vp, i64, i64, i64, vp, vp, vp, i64, i32, ctypes.POINTER(vp), vp]
    lib.tsvd_csr_create_pinned.restype = ctypes.c_int
    lib.tsvd_csr_info.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i64), ctypes.POINTER(i64)]
    lib.tsvd_csr_info.restype = ctypes.c_int
    lib.tsvd_csr_destroy.argtypes = [vp]
    lib.tsvd_csr_destroy.restype = None
    lib.tsvd_csr_get_csc.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.tsvd_csr_get_csc.restype = ctypes.c_int
    lib.tsvd_spmv.argtypes = [vp, vp, i32, vp, i32, vp, vp]
    lib.tsvd_spmv.restype = ctypes.c_int
    lib.tsvd_sparse.argtypes = [vp, vp, ctypes.POINTER(TsvdOpts), vp, i64, vp, vp, i64, ctypes.POINTER(TsvdInfo), vp]
    lib.tsvd_sparse.restype = ctypes.c_int
    _lib = lib
    return lib


def _torch():
    import torch
    return torch


class Context:
    """Owns a tsvd_ctx on one device."""

    def __init__(self, device: int = 0):
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device is visible: the t-SVD library runs on the GPU only")
        self.lib = load_library()
        self.device = device
        self.num_cu = torch.cuda.get_device_properties(device).multi_processor_count
        h = ctypes.c_void_p()
        st = self.lib.tsvd_ctx_create(device, ctypes.byref(h))
        if st != OK:
            raise TsvdError(st, f"tsvd_ctx_create({device}) failed")
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            self.lib.tsvd_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def last_error(self) -> str:
        return self.lib.tsvd_last_error(self.handle).decode()

    def check(self, st: int, allow=(OK,)):
        if st not in allow:
            raise TsvdError(st, self.last_error())
        return st


TUNING_FIELDS = ("gram_tile", "gram_chunks", "power_blocks", "team_kib", "group_kchunk", "sparse_row_bits",
                 "sparse_col_bits", "power_path")


def set_tuning(ctx: Context, gram_tile: int = 0, gram_chunks: int = 0, power_blocks: int = 0, team_kib: int = 0,
               group_kchunk: int = 0, sparse_row_bits: int = 0, sparse_col_bits: int = 0, power_path: int = 0,
               group_tile=None, group_kchunk_cls=None):
    """Set the context's launch-shape tuning (0 = library choice).
    group_tile / group_kchunk_cls: the batched Gram's unit shape per
    Gram-dimension class (gram_class), as a sequence of GRAM_CLASSES entries
    or a {class: value} dict; missing classes are 0."""
    t = TsvdTuning()
    t.gram_tile, t.gram_chunks, t.power_blocks = int(gram_tile), int(gram_chunks), int(power_blocks)
    t.team_kib, t.group_kchunk = int(team_kib), int(group_kchunk)
    t.sparse_row_bits, t.sparse_col_bits = int(sparse_row_bits), int(sparse_col_bits)
    t.power_path = int(power_path)
    for name, val in (("group_tile", group_tile), ("group_kchunk_cls", group_kchunk_cls)):
        arr = getattr(t, name)
        if val is None:
            continue
        items = val.items() if isinstance(val, dict) else enumerate(val)
        for c, v in items:
            c = int(c)
            if not 0 <= c < GRAM_CLASSES:
                raise ValueError(f"{name}: class {c} outside [0, {GRAM_CLASSES})")
            arr[c] = int(v)
    ctx.check(ctx.lib.tsvd_ctx_set_tuning(ctx.handle, ctypes.byref(t)))


def get_tuning(ctx: Context) -> dict:
    t = TsvdTuning()
    ctx.check(ctx.lib.tsvd_ctx_get_tuning(ctx.handle, ctypes.byref(t)))
    out = {f: getattr(t, f) for f in TUNING_FIELDS}
    out["group_tile"] = list(t.group_tile)
    out["group_kchunk_cls"] = list(t.group_kchunk_cls)
    return out


def _stream(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dtype_code(t) -> int:
    torch = _torch()
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.float64:
        return F64
    raise TypeError(f"A must be float32 or float64, got {t.dtype}")


def _rowmajor(A):
    if A.dim() != 2 or A.stride(1) != 1 or A.stride(0) < A.shape[1]:
        raise ValueError("A must be a 2-D row-major tensor (stride(1) == 1, stride(0) >= n)")
    return A.shape[0], A.shape[1], A.stride(0)


def _colmajor_out(rows: int, k: int, device, dtype=None):
    torch = _torch()
    t = torch.zeros((k, rows), dtype=dtype or torch.float64, device=device)
    return t.T  # rows x k, column-major


def _make_opts(lib, k, eps, v0, max_iter, fixed_iters, gram, rows_per_block, hbm_budget, branch):
    o = TsvdOpts()
    lib.tsvd_opts_default(ctypes.byref(o))
    o.k = int(k)
    o.eps = float(eps)
    o.max_iter = int(max_iter)
    keep = None
    if fixed_iters is not None:
        arr = (ctypes.c_int32 * len(fixed_iters))(*[int(x) for x in fixed_iters])
        o.fixed_iters = ctypes.cast(arr, ctypes.POINTER(ctypes.c_int32))
        keep = arr
    o.v0 = ctypes.c_void_p(v0.data_ptr()) if v0 is not None else None
    o.gram = GRAM[gram] if isinstance(gram, str) else int(gram)
    o.rows_per_block = int(rows_per_block)
    o.hbm_budget = int(hbm_budget)
    o.branch = int(branch)
    return o, keep


def _info_dict(info: TsvdInfo, it, lam, k, status):
    return {
        "status": STATUS.get(status, status),
        "k_done": info.k_done,
        "rank_deficient": bool(info.rank_deficient),
        "converged": bool(info.converged),
        "branch_right": bool(info.branch_right),
        "iters": [it[i] for i in range(k)],
        "lambda": [lam[i] for i in range(k)],
        "t_gram_ms": info.t_gram_ms,
        "t_eig_ms": info.t_eig_ms,
        "t_final_ms": info.t_final_ms,
        "t_total_ms": info.t_total_ms,
        "workspace_bytes": info.workspace_bytes,
        "h2d_bytes": info.h2d_bytes,
        "latency_ms": info.latency_ms,
        "t_stream_copy_ms": info.t_stream_copy_ms,
        "t_stream_compute_ms": info.t_stream_compute_ms,
        "t_stream_overlap_ms": info.t_stream_overlap_ms,
    }


def _check_v0(v0, k, d, device):
    torch = _torch()
    if v0 is None:
        raise ValueError("v0 (k x d start vectors, float64 on the device) is required")
    if v0.dtype != torch.float64 or v0.device != device or not v0.is_contiguous() or tuple(v0.shape) != (k, d):
        raise ValueError(f"v0 must be a contiguous float64 ({k}, {d}) tensor on {device}")


def tsvd_gram_dense(ctx: Context, A, gram="bf16x3", side="right", rows_per_block=0, B=None, accumulate=False,
                    stream=None):
    """B = A^T A (side 'right') or A A^T ('left'), both triangles, on the device."""
    torch = _torch()
    m, n, lda = _rowmajor(A)
    d = n if side == "right" else m
    gcode = GRAM[gram] if isinstance(gram, str) else int(gram)
    bdt = torch.float64 if gcode == GRAM["fp64"] or (gcode == 0 and A.dtype == torch.float64) else torch.float32
    if B is None:
        B = torch.zeros((d, d), dtype=bdt, device=A.device)
    st = ctx.lib.tsvd_gram_dense(ctx.handle, ctypes.c_void_p(A.data_ptr()), _dtype_code(A), m, n, lda, gcode,
                                 SIDE[side], int(rows_per_block), ctypes.c_void_p(B.data_ptr()), B.stride(0),
                                 1 if accumulate else 0, _stream(stream))
    ctx.check(st)
    return B


def tsvd_power_gram(ctx: Context, B, k, eps, v0, max_iter=10000, fixed_iters=None, stream=None):
    """Power iteration with deflation on the symmetric B (overwritten by the
    deflated Gram).  Returns (X [d x k] column-major float64, info)."""
    torch = _torch()
    d = B.shape[0]
    kk = d if k == -1 else k
    _check_v0(v0, kk, d, B.device)
    X = _colmajor_out(d, kk, B.device)
    o, keep = _make_opts(ctx.lib, k, eps, v0, max_iter, fixed_iters, "auto", 0, 0, 0)
    it = (ctypes.c_int32 * kk)()
    lam = (ctypes.c_double * kk)()
    info = TsvdInfo()
    info.iters = ctypes.cast(it, ctypes.POINTER(ctypes.c_int32))
    info.lambda_ = ctypes.cast(lam, ctypes.POINTER(ctypes.c_double))
    st = ctx.lib.tsvd_power_gram(ctx.handle, ctypes.c_void_p(B.data_ptr()), _dtype_code(B), d, B.stride(0),
                                 ctypes.byref(o), ctypes.c_void_p(X.data_ptr()), X.stride(1), ctypes.byref(info),
                                 _stream(stream))
    ctx.check(st, allow=(OK, NOT_CONVERGED))
    del keep
    return X, _info_dict(info, it, lam, kk, st)


def tsvd_finish_dense(ctx: Context, A, side, X, k, stream=None):
    """W = A X ('right') or A^T X ('left') in FP64, S = column norms, W /= S."""
    torch = _torch()
    m, n, lda = _rowmajor(A)
    M = m if side == "right" else n
    W = _colmajor_out(M, k, A.device)
    S = torch.zeros(k, dtype=torch.float64, device=A.device)
    if X.stride(0) != 1:
        raise ValueError("X must be column-major (stride(0) == 1)")
    st = ctx.lib.tsvd_finish_dense(ctx.handle, ctypes.c_void_p(A.data_ptr()), _dtype_code(A), m, n, lda, SIDE[side],
                                   ctypes.c_void_p(X.data_ptr()), X.stride(1), int(k), ctypes.c_void_p(W.data_ptr()),
                                   W.stride(1), ctypes.c_void_p(S.data_ptr()), _stream(stream))
    ctx.check(st)
    return W, S


def _factor_out(rows: int, k: int, device, factor: str):
    """Output for the iterated factor: on the device, or pinned host memory
    (factor="host")."""
    torch = _torch()
    if factor == "device":
        return _colmajor_out(rows, k, device)
    if factor == "host":
        return torch.zeros((k, rows), dtype=torch.float64, pin_memory=True).T
    raise ValueError('factor must be "device" or "host"')


def tsvd_dense(ctx: Context, A, k, eps, v0, max_iter=10000, fixed_iters=None, gram="auto", rows_per_block=0,
               hbm_budget=0, branch=0, stream=None, raise_not_converged=False, queue_depth=2, method="auto",
               factor="device", factor_batches=1):
    """Whole t-SVD of a dense A.  A is a device tensor (resident in HBM) or a
    pinned host tensor (``A.is_pinned()``: streamed in row batches, or in
    column batches when m < n).  method:
    "gram" (form the Gram once), "implicit" (A^T (A x) every iteration) or
    "auto".  factor="host" keeps the iterated factor (V on the right branch,
    U on the left) in pinned host memory, batched to the device in
    factor_batches row batches for every projection.  Returns (U, S, V, info),
    with U (m x k) and V (n x k) column-major float64 and S float64."""
    torch = _torch()
    m, n, lda = _rowmajor(A)
    kk = min(m, n) if k == -1 else k
    right = (m > n) if branch == 1 else (m >= n)
    d = n if right else m
    if A.is_cuda:
        loc, dev = LOC_DEVICE, A.device
    elif A.is_pinned():
        loc, dev = LOC_PINNED_HOST, torch.device("cuda", ctx.device)
    else:
        raise ValueError("A must be a device tensor or a pinned host tensor")
    _check_v0(v0, kk, d, dev)
    U = _factor_out(m, kk, dev, factor if not right else "device")
    V = _factor_out(n, kk, dev, factor if right else "device")
    S = torch.zeros(kk, dtype=torch.float64, device=dev)
    o, keep = _make_opts(ctx.lib, k, eps, v0, max_iter, fixed_iters, gram, rows_per_block, hbm_budget, branch)
    o.queue_depth = int(queue_depth)
    o.method = METHOD[method] if isinstance(method, str) else int(method)
    o.factor_loc = LOC_PINNED_HOST if factor == "host" else LOC_DEVICE
    o.factor_batches = int(factor_batches)
    it = (ctypes.c_int32 * kk)()
    lam = (ctypes.c_double * kk)()
    info = TsvdInfo()
    info.iters = ctypes.cast(it, ctypes.POINTER(ctypes.c_int32))
    info.lambda_ = ctypes.cast(lam, ctypes.POINTER(ctypes.c_double))
    st = ctx.lib.tsvd_dense(ctx.handle, ctypes.c_void_p(A.data_ptr()), _dtype_code(A), loc, m, n, lda,
                            ctypes.byref(o), ctypes.c_void_p(U.data_ptr()), U.stride(1), ctypes.c_void_p(S.data_ptr()),
                            ctypes.c_void_p(V.data_ptr()), V.stride(1), ctypes.byref(info), _stream(stream))
    ctx.check(st, allow=(OK,) if raise_not_converged else (OK, NOT_CONVERGED))
    del keep
    return U, S, V, _info_dict(info, it, lam, kk, st)


def _fill_problem(ctx: Context, q: TsvdProblem, p: dict, dev, zero_outputs: bool = True):
    """Fill a TsvdProblem from a problem dict; allocate U, S, V on `dev`
    (uninitialised when zero_outputs is False: the library clears them on its
    own stream, and a fill kernel on torch's stream would race with it)."""
    torch = _torch()
    A = p["A"]
    m, n, lda = _rowmajor(A)
    k = int(p["k"])
    kk = min(m, n) if k == -1 else k
    branch = int(p.get("branch", 0))
    right = (m > n) if branch == 1 else (m >= n)
    d = n if right else m
    _check_v0(p["v0"], kk, d, dev)
    if zero_outputs:
        U = _colmajor_out(m, kk, dev)
        V = _colmajor_out(n, kk, dev)
        S = torch.zeros(kk, dtype=torch.float64, device=dev)
    else:
        U = torch.empty((kk, m), dtype=torch.float64, device=dev).T
        V = torch.empty((kk, n), dtype=torch.float64, device=dev).T
        S = torch.empty(kk, dtype=torch.float64, device=dev)
    o, kp = _make_opts(ctx.lib, k, p["eps"], p["v0"], p.get("max_iter", 10000), p.get("fixed_iters"),
                       p.get("gram", "auto"), 0, 0, branch)
    it = (ctypes.c_int32 * kk)()
    lam = (ctypes.c_double * kk)()
    q.A = ctypes.c_void_p(A.data_ptr())
    q.dtype = _dtype_code(A)
    q.m, q.n, q.lda = m, n, lda
    q.opts = o
    q.U, q.ldu = ctypes.c_void_p(U.data_ptr()), U.stride(1)
    q.S = ctypes.c_void_p(S.data_ptr())
    q.V, q.ldv = ctypes.c_void_p(V.data_ptr()), V.stride(1)
    return U, S, V, kk, it, lam, kp


def tsvd_dense_batched(ctx: Context, problems, hbm_budget=0, stream=None, raise_errors=False):
    """Many dense t-SVDs in one pass.  `problems` is a list of dicts with keys
    A (float32 device tensor, row-major), k, eps, v0 and optionally max_iter,
    fixed_iters, gram ("auto", "fp32", "bf16x3") and branch.  Returns a list of
    (U, S, V, info) in the same order; info["status"] is each problem's
    status.  raise_errors=True raises on the first failing problem."""
    torch = _torch()
    count = len(problems)
    arr = (TsvdProblem * max(count, 1))()
    infos = (TsvdInfo * max(count, 1))()
    stats = (ctypes.c_int32 * max(count, 1))()
    keep, outs = [], []
    for i, p in enumerate(problems):
        if not p["A"].is_cuda:
            raise ValueError("batched problems take device tensors")
        U, S, V, kk, it, lam, kp = _fill_problem(ctx, arr[i], p, p["A"].device)
        infos[i].iters = ctypes.cast(it, ctypes.POINTER(ctypes.c_int32))
        infos[i].lambda_ = ctypes.cast(lam, ctypes.POINTER(ctypes.c_double))
        keep.append((kp, it, lam))
        outs.append((U, S, V, kk, it, lam))
    st = ctx.lib.tsvd_dense_batched(ctx.handle, count, arr, int(hbm_budget), infos, stats, _stream(stream))
    if raise_errors:
        ctx.check(st)
    elif st not in (OK, NOT_CONVERGED) and count and all(stats[i] == OK for i in range(count)):
        ctx.check(st)  # a failure before any problem ran (arguments, memory, HIP)
    res = []
    for i, (U, S, V, kk, it, lam) in enumerate(outs):
        res.append((U, S, V, _info_dict(infos[i], it, lam, kk, stats[i])))
    del keep
    return res


class Server:
    """A tsvd_server: continuous batching of dense requests on the context's
    device.  The context must not be used for other calls while the server
    lives.  submit() returns a ticket at once; poll()/wait() return
    (U, S, V, info) once the request completed (info["status"] holds its
    status)."""

    def __init__(self, ctx: Context, hbm_budget: int, max_slots: int = 0, max_batch: int = 0, lanes: int = 0):
        self.ctx = ctx
        cfg = TsvdServerConfig(int(hbm_budget), int(max_slots), int(max_batch), int(lanes))
        h = ctypes.c_void_p()
        ctx.check(ctx.lib.tsvd_server_create(ctx.handle, ctypes.byref(cfg), ctypes.byref(h)))
        self.handle = h
        self._live = {}  # ticket -> (outputs, references kept alive)

    def submit(self, problem: dict) -> int:
        """Queue one request (keys as for tsvd_dense_batched).  A may be a
        device tensor or a pinned host tensor (copied by the server)."""
        torch = _torch()
        A = problem["A"]
        if A.is_cuda:
            loc, dev = LOC_DEVICE, A.device
        elif A.is_pinned():
            loc, dev = LOC_PINNED_HOST, torch.device("cuda", self.ctx.device)
        else:
            raise ValueError("A must be a device tensor or a pinned host tensor")
        q = TsvdProblem()
        U, S, V, kk, it, lam, kp = _fill_problem(self.ctx, q, problem, dev, zero_outputs=False)
        t = ctypes.c_uint64()
        st = self.ctx.lib.tsvd_server_submit(self.handle, ctypes.byref(q), loc, ctypes.byref(t))
        if st != OK:
            raise TsvdError(st, self.ctx.lib.tsvd_server_last_error(self.handle).decode())
        self._live[t.value] = ((U, S, V, kk, it, lam), (problem, kp))
        return t.value

    def _result(self, ticket, info, st):
        (U, S, V, kk, it, lam), _ = self._live.pop(ticket)
        return U, S, V, _info_dict(info, it, lam, kk, st)

    def _info_for(self, ticket):
        (_, _, _, _, it, lam), _ = self._live[ticket]
        info = TsvdInfo()
        info.iters = ctypes.cast(it, ctypes.POINTER(ctypes.c_int32))
        info.lambda_ = ctypes.cast(lam, ctypes.POINTER(ctypes.c_double))
        return info

    def poll(self, ticket: int):
        """None while the request runs, else (U, S, V, info)."""
        info = self._info_for(ticket)
        done, st = ctypes.c_int32(), ctypes.c_int32()
        self.ctx.check(self.ctx.lib.tsvd_server_poll(self.handle, ticket, ctypes.byref(done), ctypes.byref(info),
                                                     ctypes.byref(st)))
        if not done.value:
            return None
        return self._result(ticket, info, st.value)

    def wait(self, ticket: int):
        info = self._info_for(ticket)
        st = self.ctx.lib.tsvd_server_wait(self.handle, ticket, ctypes.byref(info))
        return self._result(ticket, info, st)

    def last_error(self) -> str:
        return self.ctx.lib.tsvd_server_last_error(self.handle).decode()

    def stats(self) -> dict:
        s = TsvdServerStats()
        self.ctx.check(self.ctx.lib.tsvd_server_get_stats(self.handle, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in TsvdServerStats._fields_}

    def close(self):
        if getattr(self, "handle", None):
            self.ctx.lib.tsvd_server_destroy(self.handle)
            self.handle = None
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Csr:
    """A registered CSR matrix.  Device arrays are borrowed (this object keeps
    references to them) and the library adds its CSC copy and tiles in HBM.
    Pinned host arrays (``pin_memory()``) give a handle whose tiles stay in
    pinned host memory and are streamed to the device for every product
    (batch_bytes of tiles per batch, queue_depth device slots)."""

    def __init__(self, ctx: Context, rowptr, col, val, shape, stream=None, batch_bytes: int = 0,
                 queue_depth: int = 0):
        torch = _torch()
        m, n = int(shape[0]), int(shape[1])
        if rowptr.dtype != torch.int64 or col.dtype != torch.int32 or val.dtype != torch.float32:
            raise TypeError("CSR arrays must be int64 rowptr, int32 col, float32 val")
        pinned = not rowptr.is_cuda
        for t in (rowptr, col, val):
            if not t.is_contiguous() or (t.is_cuda if pinned else not t.is_cuda):
                raise ValueError("CSR arrays must be contiguous, all device tensors or all pinned host tensors")
            if pinned and not t.is_pinned():
                raise ValueError("host CSR arrays must be pinned (tensor.pin_memory())")
        if rowptr.numel() != m + 1 or col.numel() != val.numel():
            raise ValueError("rowptr must have m + 1 entries and col/val the same length")
        self.ctx, self.shape, self.nnz, self.pinned = ctx, (m, n), int(col.numel()), pinned
        self._keep = (rowptr, col, val) if not pinned else ()
        h = ctypes.c_void_p()
        ptrs = (ctypes.c_void_p(rowptr.data_ptr()), ctypes.c_void_p(col.data_ptr()), ctypes.c_void_p(val.data_ptr()))
        if pinned:
            st = ctx.lib.tsvd_csr_create_pinned(ctx.handle, m, n, self.nnz, *ptrs, int(batch_bytes), int(queue_depth),
                                                ctypes.byref(h), _stream(stream))
        else:
            st = ctx.lib.tsvd_csr_create(ctx.handle, m, n, self.nnz, *ptrs, ctypes.byref(h), _stream(stream))
        ctx.check(st)
        self.handle = h

    def info(self) -> dict:
        loc, nb, dev = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64()
        self.ctx.check(self.ctx.lib.tsvd_csr_info(self.handle, ctypes.byref(loc), ctypes.byref(nb), ctypes.byref(dev)))
        return {"loc": "pinned_host" if loc.value == LOC_PINNED_HOST else "device", "batches": nb.value,
                "device_bytes": dev.value}

    def close(self):
        if getattr(self, "handle", None):
            self.ctx.lib.tsvd_csr_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tsvd_csr_create(ctx: Context, rowptr, col, val, shape, stream=None) -> Csr:
    return Csr(ctx, rowptr, col, val, shape, stream)


def tsvd_csr_create_pinned(ctx: Context, rowptr, col, val, shape, batch_bytes=0, queue_depth=0, stream=None) -> Csr:
    """A CSR handle whose tiles stay in pinned host memory (arrays: pinned host tensors)."""
    return Csr(ctx, rowptr, col, val, shape, stream, batch_bytes, queue_depth)


def tsvd_csr_get_csc(ctx: Context, csr: Csr, stream=None):
    """(colptr int64 [n+1], rowidx int32 [nnz], val float32 [nnz]) of the CSC copy."""
    torch = _torch()
    dev = torch.device("cuda", ctx.device)
    m, n = csr.shape
    cp = torch.empty(n + 1, dtype=torch.int64, device=dev)
    ri = torch.empty(max(csr.nnz, 1), dtype=torch.int32, device=dev)
    cv = torch.empty(max(csr.nnz, 1), dtype=torch.float32, device=dev)
    st = ctx.lib.tsvd_csr_get_csc(ctx.handle, csr.handle, ctypes.c_void_p(cp.data_ptr()),
                                  ctypes.c_void_p(ri.data_ptr()), ctypes.c_void_p(cv.data_ptr()), _stream(stream))
    ctx.check(st)
    return cp, ri[: csr.nnz], cv[: csr.nnz]


def tsvd_spmv(ctx: Context, csr: Csr, x, trans: int = 0, stream=None):
    """y = A x (trans 0) or A^T x (trans 1), FP64 accumulation; x float32 or float64."""
    torch = _torch()
    m, n = csr.shape
    nin, nout = (n, m) if trans == 0 else (m, n)
    if x.numel() != nin or not x.is_cuda or not x.is_contiguous():
        raise ValueError(f"x must be a contiguous device vector of {nin} entries")
    y = torch.empty(nout, dtype=torch.float64, device=x.device)
    st = ctx.lib.tsvd_spmv(ctx.handle, csr.handle, int(trans), ctypes.c_void_p(x.data_ptr()), _dtype_code(x),
                           ctypes.c_void_p(y.data_ptr()), _stream(stream))
    ctx.check(st)
    return y


def tsvd_sparse(ctx: Context, csr: Csr, k, eps, v0, max_iter=10000, fixed_iters=None, branch=0, hbm_budget=0,
                stream=None, raise_not_converged=False, factor="device", factor_batches=1, queue_depth=2):
    """Whole t-SVD of a registered CSR matrix.  factor="host" keeps the
    iterated factor in pinned host memory (batched to the device for every
    projection, factor_batches batches through queue_depth device buffers).
    Returns (U, S, V, info)."""
    torch = _torch()
    m, n = csr.shape
    kk = min(m, n) if k == -1 else k
    right = (m > n) if branch == 1 else (m >= n)
    d = n if right else m
    dev = torch.device("cuda", ctx.device)
    _check_v0(v0, kk, d, dev)
    U = _factor_out(m, kk, dev, factor if not right else "device")
    V = _factor_out(n, kk, dev, factor if right else "device")
    S = torch.zeros(kk, dtype=torch.float64, device=dev)
    o, keep = _make_opts(ctx.lib, k, eps, v0, max_iter, fixed_iters, "auto", 0, hbm_budget, branch)
    o.queue_depth = int(queue_depth)
    o.factor_loc = LOC_PINNED_HOST if factor == "host" else LOC_DEVICE
    o.factor_batches = int(factor_batches)
    it = (ctypes.c_int32 * kk)()
    lam = (ctypes.c_double * kk)()
    info = TsvdInfo()
    info.iters = ctypes.cast(it, ctypes.POINTER(ctypes.c_int32))
    info.lambda_ = ctypes.cast(lam, ctypes.POINTER(ctypes.c_double))
    st = ctx.lib.tsvd_sparse(ctx.handle, csr.handle, ctypes.byref(o), ctypes.c_void_p(U.data_ptr()), U.stride(1),
                             ctypes.c_void_p(S.data_ptr()), ctypes.c_void_p(V.data_ptr()), V.stride(1),
                             ctypes.byref(info), _stream(stream))
    ctx.check(st, allow=(OK,) if raise_not_converged else (OK, NOT_CONVERGED))
    del keep
    return U, S, V, _info_dict(info, it, lam, kk, st)
