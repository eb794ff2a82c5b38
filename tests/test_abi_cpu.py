"""C-ABI checks that need no GPU: the library loads, exports every symbol that
include/bb.h declares, validates arguments before touching a device, and its
host-side planning and byte model agree with independent Python codings."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bb.h")

bb = pytest.importorskip("paper_2510_12705_amd.bb")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(bb_[a-z_0-9]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_expected_entry_points():
    names = _declared_functions()
    for required in ("bb_reduce", "bb_reduce_batched", "bb_set_params", "bb_autotune",
                     "bb_workspace_bytes", "bb_error_string"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(bb.LIB_PATH)
    for name in _declared_functions():
        assert hasattr(lib, name), name


def test_argument_validation_without_device():
    L = bb.lib
    vp = ctypes.c_void_p
    dummy = vp(0x1000)
    assert L.bb_reduce(-1, 4, 0, dummy, 5, dummy, dummy, None) == -1
    assert L.bb_reduce(8, -1, 0, dummy, 5, dummy, dummy, None) == -2
    assert L.bb_reduce(8, 4, 7, dummy, 5, dummy, dummy, None) == -3
    assert L.bb_reduce(8, 4, 0, None, 5, dummy, dummy, None) == -4
    assert L.bb_reduce(8, 4, 0, dummy, 4, dummy, dummy, None) == -5
    assert L.bb_reduce(8, 4, 0, dummy, 5, None, dummy, None) == -6
    assert L.bb_reduce(8, 4, 0, dummy, 5, dummy, None, None) == -7
    assert L.bb_reduce(0, 4, 0, None, 5, None, None, None) == 0     # n = 0 is a no-op
    # the allocation-free entry point validates the same arguments the same way
    assert L.bb_reduce_noalloc(-1, 4, 0, dummy, 5, dummy, dummy, None) == -1
    assert L.bb_reduce_noalloc(8, -1, 0, dummy, 5, dummy, dummy, None) == -2
    assert L.bb_reduce_noalloc(8, 4, 7, dummy, 5, dummy, dummy, None) == -3
    assert L.bb_reduce_noalloc(8, 4, 0, None, 5, dummy, dummy, None) == -4
    assert L.bb_reduce_noalloc(8, 4, 0, dummy, 4, dummy, dummy, None) == -5
    assert L.bb_reduce_noalloc(8, 4, 0, dummy, 5, None, dummy, None) == -6
    assert L.bb_reduce_noalloc(8, 4, 0, dummy, 5, dummy, None, None) == -7
    assert L.bb_reduce_noalloc(0, 4, 0, None, 5, None, None, None) == 0
    # the singular-vector entry point: the same checks plus the factors' leading dimensions
    assert L.bb_reduce_vectors(-1, 4, 0, dummy, 5, dummy, dummy, None, 0, None, 0, None) == -1
    assert L.bb_reduce_vectors(8, 4, 3, dummy, 5, dummy, dummy, None, 0, None, 0, None) == -3
    assert L.bb_reduce_vectors(8, 4, 0, dummy, 5, dummy, dummy, dummy, 7, None, 0, None) == -9
    assert L.bb_reduce_vectors(8, 4, 0, dummy, 5, dummy, dummy, None, 0, dummy, 7, None) == -11
    assert L.bb_reduce_vectors(0, 4, 0, None, 5, None, None, None, 0, None, 0, None) == 0
    I64 = ctypes.c_int64 * 1
    VP = ctypes.c_void_p * 1
    assert L.bb_reduce_batched(-1, None, None, 0, None, None, None, None, None) == -1
    assert L.bb_reduce_batched(1, I64(-3), I64(4), 0, VP(0x1000), I64(5), VP(0x1000), VP(0x1000), None) == -2
    assert L.bb_reduce_batched(1, I64(8), I64(4), 0, VP(0x1000), I64(2), VP(0x1000), VP(0x1000), None) == -6
    assert L.bb_reduce_batched(1, I64(8), I64(4), 9, VP(0x1000), I64(5), VP(0x1000), VP(0x1000), None) == -4
    assert L.bb_reduce_batched(0, None, None, 0, None, None, None, None, None) == 0
    assert L.bb_bidiag_sigma(-1, dummy, dummy, dummy, None) == -1
    assert L.bb_bidiag_sigma(4, None, dummy, dummy, None) == -2
    assert L.bb_bidiag_sigma(4, dummy, None, dummy, None) == -3
    assert L.bb_bidiag_sigma(4, dummy, dummy, None, None) == -4
    assert L.bb_bidiag_sigma(0, None, None, None, None) == 0       # n = 0 is a no-op
    assert bb.bb_error_string(-3) == "invalid argument"
    assert "watchdog" in bb.bb_error_string(2)


def test_params_roundtrip_and_rejection():
    bb.set_params(tw=8, threads_per_window=128, sweeps_per_group=4, groups_per_cu=2, lag=0, xcd_run=5)
    p = bb.get_params()
    assert (p.tw, p.threads_per_window, p.sweeps_per_group, p.groups_per_cu, p.lag, p.xcd_run) == (8, 128, 4, 2, 0, 5)
    with pytest.raises(bb.BBError):
        bb.set_params(tw=65)   # widest compiled tile is 64 (FP32 / FP16 storage)
    with pytest.raises(bb.BBError):
        bb.set_params(threads_per_window=96)
    with pytest.raises(bb.BBError):
        bb.set_params(threads_per_window=256, sweeps_per_group=8)   # 2048 threads
    with pytest.raises(bb.BBError):
        bb.set_params(xcd_run=-1)
    p2 = bb.get_params()
    assert p2.tw == 8  # a rejected call leaves the state unchanged
    bb.reset_params()
    assert bb.get_params().tw == 0


def _py_stages(b, tw):
    out = []
    while b > 1:
        t = min(tw, b - 1)
        out.append((b, t, b - t))
        b -= t
    return out


@pytest.mark.parametrize("b,tw", [(128, 16), (128, 32), (17, 16), (64, 64), (5, 1), (1, 4), (0, 4), (256, 16)])
def test_plan_matches_stage_recursion(b, tw):
    got = bb.plan(b, tw)
    exp = _py_stages(b, tw)
    assert [g[:3] for g in got] == exp
    for (bs, t, c, lag) in got:
        assert lag == bb.min_lag(c)


def test_plan_counts_named_in_the_workloads():
    assert len(bb.plan(128, 16)) == 8     # 128 -> 112 -> ... -> 16 -> 1
    assert len(bb.plan(128, 32)) == 4     # 128 -> 96 -> 64 -> 32 -> 1


def _py_model_bytes(n, b, elem, tw):
    tot = 0
    for (bs, t, c) in _py_stages(min(b, n - 1), tw):
        r = 0
        while r + c + 1 <= n - 1:
            j = 0
            while True:
                if j == 0:
                    k, p = r, r + c
                    m = min(r + bs, n - 1) - p
                else:
                    k = r + c + (j - 1) * bs
                    p = k + bs
                    m = min(t, n - 1 - p)
                if m < 1:
                    break
                L = min(p + m + bs, n - 1)
                tall = (p + m - k + 1) * (m + 1)
                wide = (m + 1) * (L - p + 1)
                tot += tall + wide - (m + 1) * (m + 1)
                j += 1
            r += 1
    return 2.0 * tot * elem


@pytest.mark.parametrize("n,b,tw,elem", [(200, 16, 4, 8), (257, 33, 16, 4), (100, 7, 16, 2), (64, 63, 8, 8)])
def test_model_bytes_matches_enumeration(n, b, tw, elem):
    assert bb.model_bytes(n, b, elem, tw) == pytest.approx(_py_model_bytes(n, b, elem, tw), rel=1e-12)


def test_model_bytes_headline_figures():
    # read + write of every step window at n = 32768, b = 128
    assert bb.model_bytes(32768, 128, 8, 16) == pytest.approx(2.71e12, rel=0.01)
    assert bb.model_bytes(32768, 128, 4, 32) == pytest.approx(1.42e12, rel=0.01)


def test_workspace_bytes_accounts_for_fill_rows():
    n, b = 1000, 64
    ws = bb.bb_workspace_bytes(n, b, bb.F64)
    assert ws >= n * (b + 2 * 16 + 1) * 8
    assert bb.bb_workspace_bytes(0, 4, bb.F64) == 0
