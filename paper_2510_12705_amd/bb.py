"""ctypes binding of the C ABI in ``include/bb.h`` (argument marshalling only).

Every step of the reduction runs in the HIP library ``lib/libbb.so``; this
module only converts torch tensors / numpy arrays into the pointers and sizes
the C functions take.  If the library is missing this module raises on import:
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "lib", "libbb.so")

F64, F32, F16 = 0, 1, 2
_ERRNAMES = {1: "BB_ERR_HIP", 2: "BB_ERR_TIMEOUT", 3: "BB_ERR_NOMEM", 4: "BB_ERR_UNSUPPORTED",
             5: "BB_ERR_NODEVICE", 6: "BB_ERR_SCRATCH"}


class BBError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__("%s failed: %d (%s)" % (where, code, _ERRNAMES.get(code, "invalid argument %d" % -code
                                                                          if code < 0 else "?")))


class Params(ctypes.Structure):
    _fields_ = [("tw", ctypes.c_int), ("threads_per_window", ctypes.c_int),
                ("sweeps_per_group", ctypes.c_int), ("groups_per_cu", ctypes.c_int), ("lag", ctypes.c_int),
                ("xcd_run", ctypes.c_int)]

    def __repr__(self):
        return "Params(tw=%d, threads_per_window=%d, sweeps_per_group=%d, groups_per_cu=%d, lag=%d, xcd_run=%d)" % (
            self.tw, self.threads_per_window, self.sweeps_per_group, self.groups_per_cu, self.lag, self.xcd_run)


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("HIP library %s is not built (run __graft_entry__.build())" % LIB_PATH)
    # torch ships its own HIP runtime under the same soname as the system one; it
    # must be loaded first so that the library binds to it and both share one
    # runtime (device memory and streams come from torch).
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    i64, vp, dp, ip = ctypes.c_int64, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)
    lib.bb_reduce.argtypes = [i64, i64, ctypes.c_int, vp, i64, vp, vp, vp]
    lib.bb_reduce.restype = ctypes.c_int
    lib.bb_reduce_vectors.argtypes = [i64, i64, ctypes.c_int, vp, i64, vp, vp, vp, i64, vp, i64, vp]
    lib.bb_reduce_vectors.restype = ctypes.c_int
    lib.bb_sym_reduce.argtypes = [i64, i64, ctypes.c_int, vp, i64, vp, vp, vp]
    lib.bb_sym_reduce.restype = ctypes.c_int
    lib.bb_sym_model_bytes.argtypes = [i64, i64, ctypes.c_int, ctypes.c_int]
    lib.bb_sym_model_bytes.restype = ctypes.c_double
    lib.bb_sym_min_lag.argtypes = [i64]
    lib.bb_sym_min_lag.restype = ctypes.c_int
    lib.bb_reduce_noalloc.argtypes = [i64, i64, ctypes.c_int, vp, i64, vp, vp, vp]
    lib.bb_reduce_noalloc.restype = ctypes.c_int
    lib.bb_reduce_batched.argtypes = [i64, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.c_int,
                                      ctypes.POINTER(vp), ctypes.POINTER(i64), ctypes.POINTER(vp),
                                      ctypes.POINTER(vp), vp]
    lib.bb_reduce_batched.restype = ctypes.c_int
    lib.bb_set_params.argtypes = [ctypes.POINTER(Params)]
    lib.bb_set_params.restype = ctypes.c_int
    lib.bb_get_params.argtypes = [ctypes.POINTER(Params)]
    lib.bb_get_params.restype = ctypes.c_int
    lib.bb_autotune.argtypes = [i64, i64, ctypes.c_int, vp, ctypes.POINTER(Params)]
    lib.bb_autotune.restype = ctypes.c_int
    lib.bb_autotune_batched.argtypes = [i64, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.c_int, vp,
                                        ctypes.POINTER(Params)]
    lib.bb_autotune_batched.restype = ctypes.c_int
    lib.bb_resolved_params.argtypes = [i64, i64, ctypes.c_int, ctypes.POINTER(Params)]
    lib.bb_resolved_params.restype = ctypes.c_int
    lib.bb_workspace_bytes.argtypes = [i64, i64, ctypes.c_int]
    lib.bb_workspace_bytes.restype = ctypes.c_size_t
    lib.bb_model_bytes.argtypes = [i64, i64, ctypes.c_int, ctypes.c_int]
    lib.bb_model_bytes.restype = ctypes.c_double
    lib.bb_plan.argtypes = [i64, ctypes.c_int, ctypes.c_int, ip, ip, ip, ip]
    lib.bb_plan.restype = ctypes.c_int
    lib.bb_min_lag.argtypes = [i64]
    lib.bb_min_lag.restype = ctypes.c_int
    lib.bb_bidiag_sigma.argtypes = [i64, vp, vp, vp, vp]
    lib.bb_bidiag_sigma.restype = ctypes.c_int
    lib.bb_stream_status.argtypes = [vp]
    lib.bb_stream_status.restype = ctypes.c_int
    lib.bb_timing_enable.argtypes = [ctypes.c_int]
    lib.bb_timing_enable.restype = ctypes.c_int
    lib.bb_timing_read.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)]
    lib.bb_timing_read.restype = ctypes.c_int
    lib.bb_release.argtypes = []
    lib.bb_release.restype = ctypes.c_int
    lib.bb_error_string.argtypes = [ctypes.c_int]
    lib.bb_error_string.restype = ctypes.c_char_p
    return lib


lib = _load()

EXPORTS = ("bb_reduce", "bb_reduce_vectors", "bb_sym_reduce", "bb_sym_min_lag", "bb_sym_model_bytes", "bb_reduce_noalloc", "bb_reduce_batched", "bb_set_params", "bb_get_params", "bb_autotune", "bb_autotune_batched", "bb_resolved_params",
           "bb_workspace_bytes", "bb_model_bytes", "bb_plan", "bb_min_lag", "bb_stream_status",
           "bb_release", "bb_error_string", "bb_timing_enable", "bb_timing_read", "bb_bidiag_sigma")


def _check(rc: int, where: str):
    if rc != 0:
        raise BBError(rc, where)


def _torch_dtype_code(t):
    import torch
    return {torch.float64: F64, torch.float32: F32, torch.float16: F16}[t.dtype]


def _stream_handle(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def bb_reduce(band, n: int, b: int, d=None, e=None, stream=None, ldband: int | None = None):
    """Reduce a device band (torch tensor of shape (n, ldband), float64/32/16,
    the column-major LAPACK upper band) to bidiagonal.  Returns (d, e) float64
    device tensors.  Asynchronous on ``stream`` (default: torch's current)."""
    import torch
    if not band.is_cuda:
        raise ValueError("band must be a device tensor")
    if not band.is_contiguous():
        raise ValueError("band must be contiguous (n, ldband)")
    ld = ldband if ldband is not None else (band.shape[1] if band.dim() == 2 else b + 1)
    if d is None:
        d = torch.empty(max(n, 1), dtype=torch.float64, device=band.device)
    if e is None:
        e = torch.empty(max(n - 1, 1), dtype=torch.float64, device=band.device)
    rc = lib.bb_reduce(n, b, _torch_dtype_code(band), ctypes.c_void_p(band.data_ptr()), ld,
                       ctypes.c_void_p(d.data_ptr()), ctypes.c_void_p(e.data_ptr()), _stream_handle(stream))
    _check(rc, "bb_reduce")
    return d[:n], e[:max(n - 1, 0)]


def bb_reduce_vectors(band, n: int, b: int, want_u: bool = True, want_v: bool = True, stream=None,
                      ldband: int | None = None):
    """Reduce a device band and form the orthogonal factors: returns (d, e, U, V)
    with U^T A V = bidiag(d, e); U and V are float64 device tensors holding the
    n x n matrices (column-major storage, viewed as the matrix; None if not
    asked for)."""
    import torch
    if not band.is_cuda:
        raise ValueError("band must be a device tensor")
    if not band.is_contiguous():
        raise ValueError("band must be contiguous (n, ldband)")
    ld = ldband if ldband is not None else (band.shape[1] if band.dim() == 2 else b + 1)
    dev = band.device
    d = torch.empty(max(n, 1), dtype=torch.float64, device=dev)
    e = torch.empty(max(n - 1, 1), dtype=torch.float64, device=dev)
    m = max(n, 1)
    Ut = torch.empty((m, m), dtype=torch.float64, device=dev) if want_u else None   # rows of Ut = columns of U
    Vt = torch.empty((m, m), dtype=torch.float64, device=dev) if want_v else None
    rc = lib.bb_reduce_vectors(n, b, _torch_dtype_code(band), ctypes.c_void_p(band.data_ptr()), ld,
                               ctypes.c_void_p(d.data_ptr()), ctypes.c_void_p(e.data_ptr()),
                               ctypes.c_void_p(Ut.data_ptr() if Ut is not None else None), m,
                               ctypes.c_void_p(Vt.data_ptr() if Vt is not None else None), m,
                               _stream_handle(stream))
    _check(rc, "bb_reduce_vectors")
    U = Ut[:n, :n].t() if Ut is not None else None
    V = Vt[:n, :n].t() if Vt is not None else None
    return d[:n], e[:max(n - 1, 0)], U, V


def bb_sym_reduce(band, n: int, b: int, d=None, e=None, stream=None, ldband: int | None = None):
    """Reduce a symmetric band (device tensor (n, ldband), float64/32, the LAPACK
    LOWER band: A(i, j) = band[j, i - j]) to tridiagonal.  Returns (d, e) float64
    device tensors: diagonal and sub-diagonal."""
    import torch
    if not band.is_cuda:
        raise ValueError("band must be a device tensor")
    if not band.is_contiguous():
        raise ValueError("band must be contiguous (n, ldband)")
    ld = ldband if ldband is not None else (band.shape[1] if band.dim() == 2 else b + 1)
    if d is None:
        d = torch.empty(max(n, 1), dtype=torch.float64, device=band.device)
    if e is None:
        e = torch.empty(max(n - 1, 1), dtype=torch.float64, device=band.device)
    rc = lib.bb_sym_reduce(n, b, _torch_dtype_code(band), ctypes.c_void_p(band.data_ptr()), ld,
                           ctypes.c_void_p(d.data_ptr()), ctypes.c_void_p(e.data_ptr()), _stream_handle(stream))
    _check(rc, "bb_sym_reduce")
    return d[:n], e[:max(n - 1, 0)]


def sym_model_bytes(n: int, b: int, elem_size: int, tw: int) -> float:
    return float(lib.bb_sym_model_bytes(n, b, elem_size, tw))


def sym_min_lag(c: int) -> int:
    return int(lib.bb_sym_min_lag(c))


def bb_reduce_noalloc(band, n: int, b: int, d, e, stream=None, ldband: int | None = None):
    """bb_reduce through the allocation-free entry point: the library works in its
    static per-device scratch.  ``d`` and ``e`` are caller-provided float64 device
    tensors (n and max(n - 1, 1) entries); returns views of them."""
    if not band.is_cuda:
        raise ValueError("band must be a device tensor")
    if not band.is_contiguous():
        raise ValueError("band must be contiguous (n, ldband)")
    ld = ldband if ldband is not None else (band.shape[1] if band.dim() == 2 else b + 1)
    rc = lib.bb_reduce_noalloc(n, b, _torch_dtype_code(band), ctypes.c_void_p(band.data_ptr()), ld,
                               ctypes.c_void_p(d.data_ptr()), ctypes.c_void_p(e.data_ptr()), _stream_handle(stream))
    _check(rc, "bb_reduce_noalloc")
    return d[:n], e[:max(n - 1, 0)]


def bidiag_sigma(d, e, sigma=None, stream=None):
    """Singular values (descending, float64 device tensor) of bidiag(d, e) given as
    float64 device tensors, computed on the device.  Asynchronous on ``stream``."""
    import torch
    n = d.shape[0]
    if sigma is None:
        sigma = torch.empty(max(n, 1), dtype=torch.float64, device=d.device)
    ep = e.data_ptr() if (e is not None and e.numel() > 0) else None
    rc = lib.bb_bidiag_sigma(n, ctypes.c_void_p(d.data_ptr()), ctypes.c_void_p(ep),
                             ctypes.c_void_p(sigma.data_ptr()), _stream_handle(stream))
    _check(rc, "bb_bidiag_sigma")
    return sigma[:n]


def bb_reduce_batched(bands, ns, bs, ds=None, es=None, stream=None):
    """Batched reduction of a list of device bands (same dtype).  Returns lists (ds, es)."""
    import torch
    count = len(bands)
    if count == 0:
        return [], []
    code = _torch_dtype_code(bands[0])
    dev = bands[0].device
    if ds is None:
        ds = [torch.empty(max(n, 1), dtype=torch.float64, device=dev) for n in ns]
    if es is None:
        es = [torch.empty(max(n - 1, 1), dtype=torch.float64, device=dev) for n in ns]
    I64 = ctypes.c_int64 * count
    VP = ctypes.c_void_p * count
    rc = lib.bb_reduce_batched(count, I64(*ns), I64(*bs), code, VP(*[t.data_ptr() for t in bands]),
                               I64(*[t.shape[1] for t in bands]), VP(*[t.data_ptr() for t in ds]),
                               VP(*[t.data_ptr() for t in es]), _stream_handle(stream))
    _check(rc, "bb_reduce_batched")
    return [x[:n] for x, n in zip(ds, ns)], [x[:max(n - 1, 0)] for x, n in zip(es, ns)]


def set_params(tw=0, threads_per_window=0, sweeps_per_group=0, groups_per_cu=0, lag=0, xcd_run=0):
    p = Params(tw, threads_per_window, sweeps_per_group, groups_per_cu, lag, xcd_run)
    _check(lib.bb_set_params(ctypes.byref(p)), "bb_set_params")


def reset_params():
    _check(lib.bb_set_params(None), "bb_set_params")


def get_params() -> Params:
    p = Params()
    _check(lib.bb_get_params(ctypes.byref(p)), "bb_get_params")
    return p


def autotune(n: int, b: int, dtype: int, stream=None) -> Params:
    p = Params()
    _check(lib.bb_autotune(n, b, dtype, _stream_handle(stream), ctypes.byref(p)), "bb_autotune")
    return p


def autotune_batched(ns, bs, dtype: int, stream=None) -> Params:
    """Tune the batched form for this exact batch of shapes (see bb.h)."""
    count = len(ns)
    I64 = ctypes.c_int64 * max(count, 1)
    p = Params()
    _check(lib.bb_autotune_batched(count, I64(*ns), I64(*bs), dtype, _stream_handle(stream), ctypes.byref(p)),
           "bb_autotune_batched")
    return p


def resolved_params(n: int, b: int, dtype: int) -> Params:
    """Launch parameters bb_reduce would use for this shape (no device work)."""
    p = Params()
    _check(lib.bb_resolved_params(n, b, dtype, ctypes.byref(p)), "bb_resolved_params")
    return p


def bb_workspace_bytes(n: int, b: int, dtype: int) -> int:
    return int(lib.bb_workspace_bytes(n, b, dtype))


def model_bytes(n: int, b: int, elem_size: int, tw: int) -> float:
    return float(lib.bb_model_bytes(n, b, elem_size, tw))


def plan(b: int, tw: int):
    """[(b_s, tw_s, c_s, lag_s)] for each stage."""
    m = 64
    arrs = [(ctypes.c_int * m)() for _ in range(4)]
    ns = lib.bb_plan(b, tw, m, *arrs)
    if ns < 0:
        raise BBError(ns, "bb_plan")
    return [tuple(a[s] for a in arrs) for s in range(min(ns, m))]


def min_lag(c: int) -> int:
    return int(lib.bb_min_lag(c))


def stream_status(stream=None) -> int:
    return int(lib.bb_stream_status(_stream_handle(stream)))


def timing_enable(on: bool = True):
    _check(lib.bb_timing_enable(1 if on else 0), "bb_timing_enable")


def timing_read():
    """(summed stage-kernel milliseconds, number of stage launches) since the last read."""
    ms = ctypes.c_double()
    cnt = ctypes.c_int64()
    _check(lib.bb_timing_read(ctypes.byref(ms), ctypes.byref(cnt)), "bb_timing_read")
    return ms.value, cnt.value


def release():
    _check(lib.bb_release(), "bb_release")


def bb_error_string(code: int) -> str:
    return lib.bb_error_string(code).decode()
