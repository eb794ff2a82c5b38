"""MI355X-native band -> bidiagonal reduction (second SVD stage).

The public API lives in :mod:`paper_2510_12705_amd.bb` (a thin ctypes binding
over the C-ABI library ``libbb.so``).  It is loaded lazily so that importing
this package for its input generators does not require the GPU library.
"""
_API = ("bb_reduce", "bb_reduce_batched", "bb_workspace_bytes", "bb_error_string", "BBError",
        "F64", "F32", "F16", "plan", "lib", "set_params", "get_params", "autotune", "model_bytes",
        "release", "Params")


def __getattr__(name):
    if name in _API:
        from . import bb
        return getattr(bb, name)
    raise AttributeError(name)
