"""The allocation-free entry point bb_reduce_noalloc, called through the C ABI.

It runs the kernels of bb_reduce in the same launch configuration with the
library's static per-device scratch as working memory, so its results must be
bitwise those of bb_reduce.  Two calls in a row, the second on a smaller band,
check that the scratch left over from a call does not leak into the next one
(counters are cleared per call; the whole working band is rewritten by pack).
"""
import ctypes
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2510_12705_amd import inputs  # noqa: E402


@pytest.fixture(scope="module")
def bb():
    from paper_2510_12705_amd import bb as _bb
    _bb.reset_params()
    yield _bb
    _bb.reset_params()


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _noalloc(bb, band, n, b, dt):
    t = torch.from_numpy(np.ascontiguousarray(band)).to("cuda:0").to(dt)
    d = torch.full((max(n, 1),), float("nan"), dtype=torch.float64, device="cuda:0")
    e = torch.full((max(n - 1, 1),), float("nan"), dtype=torch.float64, device="cuda:0")
    rc = bb.lib.bb_reduce_noalloc(n, b, bb._torch_dtype_code(t), ctypes.c_void_p(t.data_ptr()), t.shape[1],
                                  ctypes.c_void_p(d.data_ptr()), ctypes.c_void_p(e.data_ptr()),
                                  ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0, bb.bb_error_string(rc)
    st = bb.stream_status()
    assert st == 0, bb.bb_error_string(st)
    return d[:n].cpu().numpy(), e[: max(n - 1, 0)].cpu().numpy()


def _reference(bb, band, n, b, dt):
    t = torch.from_numpy(np.ascontiguousarray(band)).to("cuda:0").to(dt)
    d, e = bb.bb_reduce(t, n, b)
    assert bb.stream_status() == 0
    return d.cpu().numpy(), e.cpu().numpy()


@pytest.mark.parametrize("dt", [torch.float64, torch.float32, torch.float16])
def test_noalloc_equals_bb_reduce_on_two_calls(bb, dt):
    """Two calls in a row, the second smaller: each bitwise equal to bb_reduce."""
    for n, b, seed in ((1500, 72, 11), (333, 19, 12)):
        _say("case noalloc n=%d b=%d %s" % (n, b, dt))
        band = inputs.band_normal(n, b, seed)
        if dt == torch.float16:
            band = band * 0.25
        d1, e1 = _noalloc(bb, band, n, b, dt)
        d0, e0 = _reference(bb, band, n, b, dt)
        assert np.array_equal(d1, d0) and np.array_equal(e1, e0), (n, b, dt)


def test_noalloc_headline_shape_fits_and_matches(bb):
    """n = 32768, b = 128 FP64 (the benchmark workload) fits the scratch and is bitwise bb_reduce's."""
    n, b = 32768, 128
    _say("case noalloc n=%d b=%d fp64" % (n, b))
    assert bb.bb_workspace_bytes(n, b, bb.F64) <= 64 << 20
    band = inputs.workload("n32768_b128")
    d1, e1 = _noalloc(bb, band, n, b, torch.float64)
    d0, e0 = _reference(bb, band, n, b, torch.float64)
    assert np.array_equal(d1, d0) and np.array_equal(e1, e0)


def test_noalloc_rejects_shapes_beyond_the_scratch(bb):
    """A shape whose working memory exceeds 64 MiB returns BB_ERR_SCRATCH and leaves d, e untouched."""
    n, b = 60000, 128   # 60000 x 194 x 8 bytes of working band: above 64 MiB
    _say("case noalloc rejection n=%d b=%d" % (n, b))
    assert bb.bb_workspace_bytes(n, b, bb.F64) > 64 << 20
    band = torch.zeros((n, b + 1), dtype=torch.float64, device="cuda:0")
    d = torch.full((n,), 7.0, dtype=torch.float64, device="cuda:0")
    e = torch.full((n - 1,), 7.0, dtype=torch.float64, device="cuda:0")
    rc = bb.lib.bb_reduce_noalloc(n, b, bb.F64, ctypes.c_void_p(band.data_ptr()), b + 1,
                                  ctypes.c_void_p(d.data_ptr()), ctypes.c_void_p(e.data_ptr()),
                                  ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 6, rc
    assert "scratch" in bb.bb_error_string(rc)
    torch.cuda.synchronize()
    assert bool((d == 7.0).all()) and bool((e == 7.0).all())
    # the entry point still works after a rejected call
    d1, e1 = _noalloc(bb, inputs.band_normal(200, 9, 3), 200, 9, torch.float64)
    d0, e0 = _reference(bb, inputs.band_normal(200, 9, 3), 200, 9, torch.float64)
    assert np.array_equal(d1, d0) and np.array_equal(e1, e0)
