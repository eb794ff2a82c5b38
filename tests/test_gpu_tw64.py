"""GPU parity of the 64-wide tile (FP32 and FP16 storage; tw 33..64).

A stage whose tilewidth exceeds 32 runs the TWM = 64 kernel variant: rows and
columns of up to 65 entries, a reflector whose 65th entry is held outside the
wave's 64 lanes, two or more waves per sweep.  The oracle runs in FP64 on the
rounded input at the same tilewidth.
  * FP32 storage: max |sigma error| <= 50 n eps32 sigma_max;
  * FP16 storage: the error is measured and printed (sanity bound only);
  * launch shapes and the batched form give bitwise the same results as one
    bb_reduce in the default shape (the same per-task arithmetic).
Shapes cover tw = 64 with c = 1 (b = 65: m reaches 64, the 65th entry), the
c = 2 and c >= 3 stage kinds with a 64-wide tile, tw between 33 and 63, and
ragged tails (n not a multiple of anything).
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2510_12705_amd import inputs  # noqa: E402

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


def _gpu(bb, band, n, b, dtype, **params):
    bb.reset_params()
    bb.set_params(**params)
    t = torch.from_numpy(np.ascontiguousarray(band)).to("cuda:0").to(dtype)
    d, e = bb.bb_reduce(t, n, b)
    st = bb.stream_status()
    bb.reset_params()
    assert st == 0, bb.bb_error_string(st)
    return d.cpu().numpy(), e.cpu().numpy()


@pytest.mark.parametrize("n,b,tw", [(901, 65, 64), (1333, 64, 64), (1100, 130, 64), (777, 200, 64),
                                    (1200, 96, 48), (640, 40, 39)])
def test_fp32_tw64_sigma_error(bb, n, b, tw):
    _say("case fp32 n=%d b=%d tw=%d" % (n, b, tw))
    band32 = inputs.band_normal(n, b, seed=n + b).astype(np.float32).astype(np.float64)
    d, e = _gpu(bb, band32, n, b, torch.float32, tw=tw)
    assert d[0] == band32[0, b]
    do, eo = oracle.reduce(band32, n, b, tw)
    s_g = oracle.singular_values(d, e)
    s_o = oracle.singular_values(do, eo)
    err = np.max(np.abs(s_g - s_o))
    _say("  fp32 tw=%d sigma err %.3e = %.3f n eps32 sigma_max" % (tw, err, err / (n * EPS32 * s_o[0])))
    assert err <= 50 * n * EPS32 * s_o[0]


@pytest.mark.parametrize("n,b,tw", [(1333, 64, 64), (1100, 130, 64), (901, 65, 64)])
def test_fp16_tw64_sigma_error_measured(bb, n, b, tw):
    _say("case fp16 n=%d b=%d tw=%d" % (n, b, tw))
    band16 = inputs.band_uniform(n, b, seed=n + 7).astype(np.float16).astype(np.float64)
    d, e = _gpu(bb, band16, n, b, torch.float16, tw=tw)
    assert np.isfinite(d).all() and np.isfinite(e).all()
    do, eo = oracle.reduce(band16, n, b, tw)
    s_g = oracle.singular_values(d, e)
    s_o = oracle.singular_values(do, eo)
    rel2 = np.linalg.norm(s_g - s_o) / np.linalg.norm(s_o)
    _say("  fp16 tw=%d: max|dsigma|/sigma_max = %.3e, ||dsigma||/||sigma|| = %.3e"
         % (tw, np.max(np.abs(s_g - s_o)) / s_o[0], rel2))
    assert rel2 <= 5e-2


@pytest.mark.parametrize("params", [dict(threads_per_window=128), dict(threads_per_window=256),
                                    dict(threads_per_window=128, sweeps_per_group=2), dict(groups_per_cu=1),
                                    dict(xcd_run=5), dict(threads_per_window=64)])
def test_tw64_launch_shapes_bitwise(bb, params):
    """Every launch shape computes the same per-task arithmetic; threads_per_window
    = 64 is raised to 128 for the 64-wide stages."""
    n, b = 1157, 130
    _say("case fp32 tw=64 shape %r" % (params,))
    band = inputs.band_normal(n, b, seed=9)
    d0, e0 = _gpu(bb, band, n, b, torch.float32, tw=64)
    d1, e1 = _gpu(bb, band, n, b, torch.float32, tw=64, **params)
    assert np.array_equal(d0, d1) and np.array_equal(e0, e1)


def test_tw64_rejected_for_fp64(bb):
    n, b = 300, 70
    t = torch.from_numpy(inputs.band_normal(n, b, seed=1)).cuda()
    bb.reset_params()
    bb.set_params(tw=64)
    with pytest.raises(bb.BBError) as ei:
        bb.bb_reduce(t, n, b)
    bb.reset_params()
    assert ei.value.code == 4


@pytest.mark.parametrize("dtype", [torch.float32, torch.float16])
def test_tw64_batched_equals_individual_calls(bb, dtype):
    _say("case ragged batch tw=64 %s" % dtype)
    rng = np.random.default_rng(21)
    mats = []
    for _ in range(20):
        n = int(rng.integers(70, 900))
        b = int(rng.choice([16, 33, 64, 65, 100]))
        bd = inputs.band_uniform(n, b, seed=int(rng.integers(1 << 30)))
        mats.append((n, b, bd))
    bb.reset_params()
    bb.set_params(tw=64)
    bands = [torch.from_numpy(np.ascontiguousarray(bd)).cuda().to(dtype) for (_, _, bd) in mats]
    ns = [m[0] for m in mats]
    bs = [m[1] for m in mats]
    ds, es = bb.bb_reduce_batched(bands, ns, bs)
    assert bb.stream_status() == 0
    for t, n, b, dd, ee in zip(bands, ns, bs, ds, es):
        d1, e1 = bb.bb_reduce(t, n, b)
        assert np.array_equal(dd.cpu().numpy(), d1.cpu().numpy()), (n, b)
        assert np.array_equal(ee.cpu().numpy(), e1.cpu().numpy()), (n, b)
    bb.reset_params()
