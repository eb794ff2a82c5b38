"""The timed autotuner never makes a call slower than its defaults.

bb_autotune (one band) and bb_autotune_batched (one exact batch) time the
defaults and the other candidates three times each and keep the defaults
unless a candidate's median is at least 1 % faster.  Measured afterwards, a
call with the cached winner must take at most 1.02 x the default time
(timing noise allowance), on the n = 32768, b = 128 FP64 workload and on the
512-band ragged FP32 batch; the tuned results are still checked (FP64 bitwise
against the stored oracle hash at the chosen tilewidth; the batch bitwise
against single calls with the same parameters).
"""
import sys
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2510_12705_amd import inputs  # noqa: E402
from tests import oracle_pool  # noqa: E402


@pytest.fixture(scope="module")
def bb():
    from paper_2510_12705_amd import bb as _bb
    _bb.release()
    _bb.reset_params()
    yield _bb
    _bb.release()
    _bb.reset_params()


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _best_ms(fn, reps=3):
    fn()
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        t = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t)
    return best * 1e3


def test_autotune_single_band_not_slower_than_defaults(bb):
    n, b = 32768, 128
    _say("case autotune n=%d b=%d fp64" % (n, b))
    bb.release()
    bb.reset_params()
    band = inputs.workload("n32768_b128")
    t = torch.from_numpy(band).cuda()
    d = torch.empty(n, dtype=torch.float64, device="cuda")
    e = torch.empty(n, dtype=torch.float64, device="cuda")
    t_def = _best_ms(lambda: bb.bb_reduce(t, n, b, d, e), reps=2)
    p = bb.autotune(n, b, bb.F64)
    q = bb.resolved_params(n, b, bb.F64)
    assert (q.tw, q.threads_per_window, q.sweeps_per_group, q.groups_per_cu, q.xcd_run) == \
        (p.tw, p.threads_per_window, p.sweeps_per_group, p.groups_per_cu, p.xcd_run)
    t_tuned = _best_ms(lambda: bb.bb_reduce(t, n, b, d, e), reps=2)
    _say("  defaults %.1f ms, tuned %.1f ms with %r" % (t_def, t_tuned, p))
    assert bb.stream_status() == 0
    assert t_tuned <= 1.02 * t_def
    rec, _ = oracle_pool.golden("n32768_b128_f64_tw%d" % p.tw)
    if rec is not None:
        assert oracle_pool.de_hash(d.cpu().numpy(), e[: n - 1].cpu().numpy()) == rec["de_sha256"]
    else:
        assert d[0].item() == band[0, b]
    bb.release()


def test_autotune_batched_not_slower_than_defaults(bb):
    _say("case autotune 512 ragged fp32 batch")
    bb.release()
    bb.reset_params()
    mats = inputs.ragged_batch(count=512, seed=5)
    bands = [torch.from_numpy(np.ascontiguousarray(bd)).cuda().to(torch.float32) for (_, _, bd) in mats]
    ns = [m[0] for m in mats]
    bs = [m[1] for m in mats]
    ds = [torch.empty(max(x, 1), dtype=torch.float64, device="cuda") for x in ns]
    es = [torch.empty(max(x, 1), dtype=torch.float64, device="cuda") for x in ns]
    t_def = _best_ms(lambda: bb.bb_reduce_batched(bands, ns, bs, ds=ds, es=es))
    p = bb.autotune_batched(ns, bs, bb.F32)
    t_tuned = _best_ms(lambda: bb.bb_reduce_batched(bands, ns, bs, ds=ds, es=es))
    _say("  defaults %.1f ms, tuned %.1f ms with %r" % (t_def, t_tuned, p))
    assert bb.stream_status() == 0
    assert t_tuned <= 1.02 * t_def
    # the tuned batch computes what single calls with the same tilewidth compute
    bb.set_params(tw=p.tw)
    for i in range(0, 512, 51):
        d1, e1 = bb.bb_reduce(bands[i], ns[i], bs[i])
        assert np.array_equal(ds[i][: ns[i]].cpu().numpy(), d1.cpu().numpy()), i
        assert np.array_equal(es[i][: ns[i] - 1].cpu().numpy(), e1.cpu().numpy()), i
    bb.reset_params()
    bb.release()
