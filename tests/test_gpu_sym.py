"""GPU parity of the symmetric band -> tridiagonal reduction (bb_sym_reduce).

FP64 storage: the kernel performs the oracle's operations in the oracle's
order (one reflector per step, left pass then right pass over the mirrored
diagonal block, sequential dots without fused multiply-add) and concurrently
running steps touch disjoint entries, so d and e equal the oracle's bitwise.
FP32 storage: eigenvalues within 50 n eps32 ||A||_2 of the FP64 oracle's on the
rounded input.  Edge cases: b = 0, b = 1, b >= n, n <= 2, every stage kind
(c = 1, c = 2, c >= 3) and several tilewidths, launch shapes.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle  # noqa: E402

EPS64 = np.finfo(np.float64).eps
EPS32 = np.finfo(np.float32).eps


@pytest.fixture(scope="module")
def bb():
    from paper_2510_12705_amd import bb as _bb
    _bb.reset_params()
    yield _bb
    _bb.reset_params()


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def sym_band(n, b, seed):
    rng = np.random.default_rng(seed)
    band = rng.standard_normal((n, b + 1))
    for j in range(n):
        band[j, max(0, n - j):] = 0.0
    return band


def _gpu(bb, band, n, b, dt=torch.float64, **params):
    bb.reset_params()
    if params:
        bb.set_params(**params)
    t = torch.from_numpy(np.ascontiguousarray(band)).to("cuda:0").to(dt)
    d, e = bb.bb_sym_reduce(t, n, b)
    st = bb.stream_status()
    bb.reset_params()
    assert st == 0, bb.bb_error_string(st)
    return d.cpu().numpy(), e.cpu().numpy()


# (600, 128, 32) starts with 512-thread stages (b > 64) and ends with 256-thread ones;
# (700, 300, 16) makes both groups of a 512-thread workgroup loop (b - 1 > 256 columns, b > 192 rows)
@pytest.mark.parametrize("n,b,tw", [(512, 32, 32), (700, 40, 16), (333, 17, 4), (257, 9, 8), (200, 3, 2), (150, 2, 1),
                                    (400, 64, 32), (301, 100, 24), (90, 89, 8), (1025, 48, 32), (600, 128, 32),
                                    (700, 300, 16)])
def test_fp64_bitwise_oracle(bb, n, b, tw):
    _say("case sym fp64 n=%d b=%d tw=%d" % (n, b, tw))
    band = sym_band(n, b, seed=n + b)
    d, e = _gpu(bb, band, n, b, tw=tw)
    do, eo = oracle.sym_reduce(band, n, b, tw)
    assert np.array_equal(d, do) and np.array_equal(e, eo), (np.flatnonzero(d != do)[:4], np.flatnonzero(e != eo)[:4])


def test_default_launch_and_shapes_bitwise(bb):
    n, b = 2000, 64
    _say("case sym fp64 n=%d b=%d launch shapes" % (n, b))
    band = sym_band(n, b, seed=4)
    tw = 32
    do, eo = oracle.sym_reduce(band, n, b, tw)
    for params in ({}, {"groups_per_cu": 1}, {"groups_per_cu": 4}, {"lag": 5}):
        d, e = _gpu(bb, band, n, b, **params)
        assert np.array_equal(d, do) and np.array_equal(e, eo), params


def test_edge_cases(bb):
    for (n, b) in [(1, 0), (1, 3), (2, 1), (2, 5), (3, 2), (6, 0), (7, 1), (40, 39)]:
        band = sym_band(n, b, seed=n * 10 + b)
        d, e = _gpu(bb, band, n, b)
        do, eo = oracle.sym_reduce(band, n, b, 32)
        assert np.array_equal(d, do) and np.array_equal(e, eo), (n, b)


def test_fp32_storage_eigenvalue_error(bb):
    n, b = 1500, 64
    _say("case sym fp32 n=%d b=%d" % (n, b))
    band = sym_band(n, b, seed=8).astype(np.float32).astype(np.float64)
    d, e = _gpu(bb, band, n, b, dt=torch.float32)
    do, eo = oracle.sym_reduce(band, n, b, 32)
    w_g = oracle.sym_eigenvalues(d, e)
    w_o = oracle.sym_eigenvalues(do, eo)
    nrm = np.abs(w_o).max()
    err = np.abs(w_g - w_o).max()
    _say("  fp32 eigenvalue error %.3e = %.4f n eps32 ||A||_2" % (err, err / (n * EPS32 * nrm)))
    assert err <= 50 * n * EPS32 * nrm


def test_fp16_is_rejected(bb):
    t = torch.zeros((10, 3), dtype=torch.float16, device="cuda:0")
    with pytest.raises(bb.BBError) as ei:
        bb.bb_sym_reduce(t, 10, 2)
    assert ei.value.code == 4
