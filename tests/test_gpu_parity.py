"""GPU parity: the HIP path through the C ABI against the CPU oracle.

FP64 storage: the GPU kernels perform the oracle's arithmetic operation for
operation (same sequential dot order, no fused multiply-add, the same LAPACK
reflector formulas with correctly rounded division and square root), and
concurrently running tasks touch disjoint data, so d and e must equal the
oracle's BITWISE.  That meets the FP64 bar for (|d|, |e|) (1e-12 ||A||_F in
2-norm) with zero difference, and sigma (computed from both by the same
routine) trivially within 20 n eps64 sigma_max; both are still computed and
asserted so a failure reports magnitudes.
FP32 storage: max |sigma error| <= 50 n eps32 sigma_max against the FP64 oracle
of the FP32-rounded input.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2510_12705_amd import inputs  # noqa: E402
from tests.pins import band_to_dense, dense_to_band  # noqa: E402

EPS64 = np.finfo(np.float64).eps
EPS32 = np.finfo(np.float32).eps


@pytest.fixture(scope="module")
def bb():
    from paper_2510_12705_amd import bb as _bb
    yield _bb
    _bb.reset_params()


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_reduce(bb, band, n, b, dtype=torch.float64, **params):
    bb.reset_params()
    if params:
        bb.set_params(**params)
    t = torch.from_numpy(np.ascontiguousarray(band)).to("cuda:0").to(dtype)
    d, e = bb.bb_reduce(t, n, b)
    st = bb.stream_status()
    assert st == 0, bb.bb_error_string(st)
    return d.cpu().numpy(), e.cpu().numpy()


def check_fp64(band, n, b, tw, d, e):
    do, eo = oracle.reduce(band, n, b, tw)
    normA = np.sqrt(np.sum(band * band))
    de = np.sqrt(np.sum((np.abs(d) - np.abs(do)) ** 2) + np.sum((np.abs(e) - np.abs(eo)) ** 2))
    s_g = oracle.singular_values(d, e)
    s_o = oracle.singular_values(do, eo)
    serr = np.max(np.abs(s_g - s_o)) if n else 0.0
    first = np.flatnonzero((d != do)).tolist()[:3] + ["e"] + np.flatnonzero((e != eo)).tolist()[:3]
    assert de <= 1e-12 * normA, ("|d|,|e| 2-norm difference", de, normA, first)
    assert serr <= 20 * n * EPS64 * max(s_o[0], 1e-300), ("sigma", serr, s_o[0])
    assert np.array_equal(d, do) and np.array_equal(e, eo), ("not bitwise equal", first)
    return serr, de


def test_c1_fp64_parity(bb):
    n, b, tw = 512, 32, 16
    _say("case n=512 b=32 fp64")
    band = inputs.band_normal(n, b, seed=1)
    d, e = gpu_reduce(bb, band, n, b, tw=tw)
    check_fp64(band, n, b, tw, d, e)
    A = band_to_dense(band, n, b)
    assert d[0] == A[0, 0]


RAGGED = [(300, 17, 4), (1000, 40, 16), (777, 64, 16), (1500, 100, 32), (129, 128, 16), (96, 200, 8),
          (2049, 33, 16), (640, 9, 8), (513, 2, 1), (700, 3, 2), (333, 64, 1)]


@pytest.mark.parametrize("n,b,tw", RAGGED)
def test_ragged_fp64_parity(bb, n, b, tw):
    _say("case n=%d b=%d tw=%d fp64" % (n, b, tw))
    band = inputs.band_normal(n, b, seed=n + b)
    d, e = gpu_reduce(bb, band, n, b, tw=tw)
    check_fp64(band, n, b, tw, d, e)


@pytest.mark.parametrize("ntl,lanes", [(64, 1), (64, 4), (128, 2), (128, 8), (256, 1), (256, 4)])
def test_thread_and_lane_counts_are_bitwise_identical(bb, ntl, lanes):
    """Every thread count and group size computes the same per-row/per-column arithmetic."""
    n, b, tw = 700, 48, 16
    band = inputs.band_normal(n, b, seed=3)
    ref = gpu_reduce(bb, band, n, b, tw=tw, threads_per_window=128, sweeps_per_group=1)
    d, e = gpu_reduce(bb, band, n, b, tw=tw, threads_per_window=ntl, sweeps_per_group=lanes)
    assert np.array_equal(d, ref[0]) and np.array_equal(e, ref[1])


@pytest.mark.parametrize("ntl,lanes", [(64, 4), (128, 2), (256, 1), (256, 4), (64, 1), (128, 1)])
def test_tw32_group_shapes_are_bitwise_identical(bb, ntl, lanes):
    """The widest kernel variant (tw 17..32) takes at most 256 threads per workgroup;
    larger requested groups are reduced by the host, never changing a bit.  With one
    sweep per workgroup and 64 or 128 threads the windows (up to 112 rows / columns)
    exceed the threads, so the two-part wait meets multi-row and multi-block tasks."""
    n, b, tw = 900, 80, 32
    band = inputs.band_normal(n, b, seed=6)
    ref = gpu_reduce(bb, band, n, b, tw=tw, threads_per_window=256, sweeps_per_group=1)
    d, e = gpu_reduce(bb, band, n, b, tw=tw, threads_per_window=ntl, sweeps_per_group=lanes)
    assert np.array_equal(d, ref[0]) and np.array_equal(e, ref[1])
    check_fp64(band, n, b, tw, d, e)


@pytest.mark.parametrize("gpc,lanes", [(1, 1), (2, 3), (16, 2), (1, 8)])
def test_schedule_independence_bitwise(bb, gpc, lanes):
    """Race detector: concurrently running tasks are disjoint, so how many sweeps are in
    flight (groups per CU, sweeps per group) must not change a single bit."""
    n, b, tw = 3000, 64, 16
    band = inputs.band_normal(n, b, seed=4)
    ref = gpu_reduce(bb, band, n, b, tw=tw)
    again = gpu_reduce(bb, band, n, b, tw=tw)
    assert np.array_equal(again[0], ref[0]) and np.array_equal(again[1], ref[1])
    d, e = gpu_reduce(bb, band, n, b, tw=tw, groups_per_cu=gpc, sweeps_per_group=lanes)
    assert np.array_equal(d, ref[0]) and np.array_equal(e, ref[1])


@pytest.mark.parametrize("xcd_run", [1, 3, 64])
def test_xcd_run_is_bitwise_identical(bb, xcd_run):
    """Placement of sweep groups on XCDs (and the cache scope of the hand-over it
    implies) does not change a bit of the result."""
    n, b, tw = 1500, 48, 16
    _say("case n=%d b=%d xcd_run=%d" % (n, b, xcd_run))
    band = inputs.band_normal(n, b, seed=21)
    d, e = gpu_reduce(bb, band, n, b, tw=tw, xcd_run=xcd_run)
    do, eo = oracle.reduce(band, n, b, tw)
    assert np.array_equal(d, do) and np.array_equal(e, eo)


@pytest.mark.parametrize("n,b,tw", [(333, 64, 1), (800, 40, 2), (513, 2, 1)])
@pytest.mark.parametrize("params", [dict(), dict(groups_per_cu=1), dict(xcd_run=2), dict(threads_per_window=256)])
def test_one_sweep_per_workgroup_bitwise(bb, n, b, tw, params):
    """One sweep per workgroup hands every sweep over between workgroups, with
    tiny windows (tw <= 2) the hand-overs are microseconds apart: the results
    must still be bitwise the oracle's."""
    _say("case n=%d b=%d tw=%d one sweep per workgroup %s" % (n, b, tw, params))
    band = inputs.band_normal(n, b, seed=n + b)
    d, e = gpu_reduce(bb, band, n, b, tw=tw, sweeps_per_group=1, **params)
    do, eo = oracle.reduce(band, n, b, tw)
    assert np.array_equal(d, do) and np.array_equal(e, eo)


def test_autotune_caches_a_winner_and_results_stay_bitwise(bb):
    """The timed search returns a valid launch shape, bb_reduce then uses the
    cached entry, and the result is still the oracle's bit for bit."""
    n, b = 2048, 64
    _say("case autotune n=%d b=%d" % (n, b))
    bb.release()
    bb.reset_params()
    bb.set_params(tw=16)
    p = bb.autotune(n, b, bb.F64)
    assert p.tw == 16 and p.threads_per_window in (64, 128, 256) and p.sweeps_per_group >= 1
    q = bb.resolved_params(n, b, bb.F64)
    assert (q.tw, q.threads_per_window, q.sweeps_per_group, q.groups_per_cu) == \
        (p.tw, p.threads_per_window, p.sweeps_per_group, p.groups_per_cu)
    band = inputs.band_normal(n, b, seed=77)
    t = torch.from_numpy(band).cuda()
    d, e = bb.bb_reduce(t, n, b)
    assert bb.stream_status() == 0
    do, eo = oracle.reduce(band, n, b, 16)
    assert np.array_equal(d.cpu().numpy(), do) and np.array_equal(e.cpu().numpy(), eo)
    bb.release()
    bb.reset_params()


def test_larger_lag_is_bitwise_identical(bb):
    n, b, tw = 1200, 40, 8
    band = inputs.band_normal(n, b, seed=5)
    ref = gpu_reduce(bb, band, n, b, tw=tw)
    d, e = gpu_reduce(bb, band, n, b, tw=tw, lag=6)
    assert np.array_equal(d, ref[0]) and np.array_equal(e, ref[1])


def test_edge_cases(bb):
    _say("case edge sizes")
    # n = 1
    d, e = gpu_reduce(bb, np.array([[0.0, 0.0, 2.5]]), 1, 2)
    assert d.tolist() == [2.5]
    # n = 2, b = 1
    d, e = gpu_reduce(bb, np.array([[0.0, 1.0], [2.0, 3.0]]), 2, 1)
    assert d.tolist() == [1.0, 3.0] and e.tolist() == [2.0]
    # b = 0
    d, e = gpu_reduce(bb, np.arange(1.0, 8.0).reshape(7, 1), 7, 0)
    assert d.tolist() == [1, 2, 3, 4, 5, 6, 7] and e.tolist() == [0] * 6
    # b >= n clamps
    n = 20
    band = inputs.band_normal(n, 30, seed=6)
    d, e = gpu_reduce(bb, band, n, 30, tw=8)
    s = oracle.singular_values(d, e)
    assert np.max(np.abs(s - np.linalg.svd(band_to_dense(band, n, 30), compute_uv=False))) <= 1e-13 * s[0]
    # ldband > b + 1 (padded input)
    n, b = 300, 20
    band = inputs.band_normal(n, b, seed=7)
    padded = np.zeros((n, b + 5))
    padded[:, : b + 1] = band
    d1, e1 = gpu_reduce(bb, band, n, b, tw=8)
    bb.set_params(tw=8)
    t = torch.from_numpy(padded).cuda()
    d2, e2 = bb.bb_reduce(t, n, b)
    assert np.array_equal(d2.cpu().numpy(), d1) and np.array_equal(e2.cpu().numpy(), e1)


def test_tiny_bands_with_fewer_sweep_groups_than_xcds(bb):
    """Bands with fewer sweep groups than the device has XCDs launch fewer workgroups
    than XCDs; they must still process every group.  Workgroups of small launches land
    on XCDs that depend on the launches before them, so each case follows a device
    kernel of a different size."""
    _say("case tiny bands, varied dispatch history")
    bb.reset_params()
    rng = np.random.default_rng(17)
    for trial in range(40):
        n = int(rng.integers(3, 14))
        b = int(rng.integers(2, n + 2))
        band = inputs.band_normal(n, b, seed=100 + trial)
        _ = torch.ones(int(rng.integers(1, 64)) * 256 * 7, device="cuda").sum()  # a launch of another size
        d, e = gpu_reduce(bb, band, n, b)
        do, eo = oracle.reduce(band, n, b, bb.resolved_params(n, b, bb.F64).tw)
        assert np.array_equal(d, do) and np.array_equal(e, eo), (trial, n, b)


@pytest.mark.parametrize("n,b,tw", [(200, 8, 3), (500, 33, 16)])
def test_bidiagonal_input_unchanged(bb, n, b, tw):
    rng = np.random.default_rng(11)
    A = np.diag(rng.standard_normal(n)) + np.diag(rng.standard_normal(n - 1), 1)
    band = dense_to_band(A, b)
    d, e = gpu_reduce(bb, band, n, b, tw=tw)
    assert np.array_equal(d, np.diag(A)) and np.array_equal(e, np.diag(A, 1))


def test_tiny_scale_takes_rescaling_branch(bb):
    """A band scaled by 2^-1000 drives every reflector through the |beta| < safmin
    rescaling branch (and produces subnormal intermediates); the GPU must still
    reproduce the oracle bitwise."""
    n, b, tw = 400, 24, 16
    band = inputs.band_normal(n, b, seed=8)
    band[:, b] += 3.0 * np.sqrt(b + 1)
    band *= 2.0 ** -1000
    d, e = gpu_reduce(bb, band, n, b, tw=tw)
    assert np.isfinite(d).all() and np.isfinite(e).all()
    do, eo = oracle.reduce(band, n, b, tw)
    assert np.array_equal(d, do) and np.array_equal(e, eo)


@pytest.mark.parametrize("tw", [16, 32])
def test_huge_scale_takes_general_norm_branch(bb, tw):
    """A band scaled by 2^600 puts every nonzero entry above xNRM2's 2^486 threshold,
    so every reflector norm takes the general (scaled-accumulator) path of the device
    norm; the GPU must reproduce the oracle bitwise, and d, e must be exactly 2^600
    times those of the unscaled band."""
    n, b = 400, 24
    _say("case huge scale n=%d b=%d tw=%d" % (n, b, tw))
    band = inputs.band_normal(n, b, seed=8)
    band[:, b] += 3.0 * np.sqrt(b + 1)
    d0, e0 = gpu_reduce(bb, band, n, b, tw=tw)
    s = 2.0 ** 600
    d, e = gpu_reduce(bb, band * s, n, b, tw=tw)
    assert np.isfinite(d).all() and np.isfinite(e).all()
    do, eo = oracle.reduce(band * s, n, b, tw)
    assert np.array_equal(d, do) and np.array_equal(e, eo)
    assert np.array_equal(d, d0 * s) and np.array_equal(e, e0 * s)


def test_c2_fp64_parity(bb):
    n, b, tw = 8192, 64, 16
    _say("case n=8192 b=64 fp64 (oracle ~15 s)")
    band = inputs.workload("n8192_b64")
    d, e = gpu_reduce(bb, band, n, b, tw=tw)
    serr, de = check_fp64(band, n, b, tw, d, e)
    _say("  sigma err %.3e  |d,e| err %.3e" % (serr, de))


def test_c2_graded_fp64_parity(bb):
    n, b, tw = 8192, 64, 16
    _say("case n=8192 b=64 graded fp64")
    band = inputs.workload("n8192_b64_graded")
    d, e = gpu_reduce(bb, band, n, b, tw=tw)
    check_fp64(band, n, b, tw, d, e)


@pytest.mark.parametrize("n,b,tw", [(512, 32, 32), (1000, 40, 16), (2000, 64, 32)])
def test_fp32_storage_sigma_error(bb, n, b, tw):
    _say("case n=%d b=%d fp32" % (n, b))
    band = inputs.band_normal(n, b, seed=n)
    band32 = band.astype(np.float32).astype(np.float64)
    d, e = gpu_reduce(bb, band32, n, b, dtype=torch.float32, tw=tw)
    do, eo = oracle.reduce(band32, n, b, tw)
    s_g = oracle.singular_values(d, e)
    s_o = oracle.singular_values(do, eo)
    err = np.max(np.abs(s_g - s_o))
    _say("  fp32 sigma err %.3e = %.3f n eps32 sigma_max" % (err, err / (n * EPS32 * s_o[0])))
    assert err <= 50 * n * EPS32 * s_o[0]


@pytest.mark.parametrize("n,b,tw", [(512, 32, 32), (2000, 64, 32), (1500, 100, 16)])
def test_fp16_storage_sigma_error_measured(bb, n, b, tw):
    """FP16 storage with a per-stage power-of-two scale: the error is measured and
    reported (no target is set for it); the bound asserted is only a sanity check."""
    band = inputs.band_uniform(n, b, seed=n + 1)
    band16 = band.astype(np.float16).astype(np.float64)
    d, e = gpu_reduce(bb, band16, n, b, dtype=torch.float16, tw=tw)
    assert np.isfinite(d).all() and np.isfinite(e).all()
    do, eo = oracle.reduce(band16, n, b, tw)
    s_g = oracle.singular_values(d, e)
    s_o = oracle.singular_values(do, eo)
    rel2 = np.linalg.norm(s_g - s_o) / np.linalg.norm(s_o)
    _say("  fp16 n=%d b=%d: max|dsigma|/sigma_max = %.3e, ||dsigma||/||sigma|| = %.3e"
         % (n, b, np.max(np.abs(s_g - s_o)) / s_o[0], rel2))
    assert rel2 <= 5e-2


def test_fp16_scale_handles_tiny_and_large_inputs(bb):
    """The per-stage scale keeps FP16 storage usable for bands far from unit size."""
    n, b, tw = 600, 32, 16
    base = inputs.band_uniform(n, b, seed=12)
    res = []
    for scale in (2.0 ** -14, 1.0, 2.0 ** 10):
        band16 = (base * scale).astype(np.float16).astype(np.float64)
        d, e = gpu_reduce(bb, band16, n, b, dtype=torch.float16, tw=tw)
        assert np.isfinite(d).all() and np.isfinite(e).all()
        res.append(oracle.singular_values(d, e) / scale)
    assert np.max(np.abs(res[0] - res[1])) <= 2e-2 * res[1][0]
    assert np.max(np.abs(res[2] - res[1])) <= 2e-2 * res[1][0]


# ------------------------------------------------------------------ sigma of the bidiagonal on the device
def _gpu_sigma(bb, d, e):
    dt = torch.from_numpy(np.ascontiguousarray(d, dtype=np.float64)).cuda()
    et = torch.from_numpy(np.ascontiguousarray(e, dtype=np.float64)).cuda()
    s = bb.bidiag_sigma(dt, et)
    torch.cuda.synchronize()
    return s.cpu().numpy()


def _check_sigma(bb, d, e):
    n = len(d)
    s_gpu = _gpu_sigma(bb, d, e)
    s_ref = oracle.singular_values(d, e)
    assert np.all(np.diff(s_gpu) <= 0) and np.all(s_gpu >= 0)
    tol = 20 * n * EPS64 * max(s_ref[0], 1e-300)
    assert np.max(np.abs(s_gpu - s_ref)) <= tol, (np.max(np.abs(s_gpu - s_ref)), tol)
    return s_gpu, s_ref


@pytest.mark.parametrize("n,seed", [(1, 1), (2, 2), (3, 3), (100, 4), (1000, 5), (4097, 6)])
def test_bidiag_sigma_matches_oracle(bb, n, seed):
    """sigma(bidiag(d, e)) by bisection on the device against the oracle's LAPACK
    dsterf on the same Golub-Kahan tridiagonal."""
    _say("case bidiag sigma n=%d" % n)
    rng = np.random.default_rng(seed)
    d = rng.standard_normal(n)
    e = rng.standard_normal(max(n - 1, 0))
    _check_sigma(bb, d, e)


def test_bidiag_sigma_special_cases(bb):
    """Diagonal input (sigma = sorted |d|, exactly up to the bisection width), zeros,
    a graded spectrum and a 2 x 2 closed form."""
    _say("case bidiag sigma special cases")
    d = np.array([3.0, -1.0, 0.0, 2.0, -7.5])
    s = _gpu_sigma(bb, d, np.zeros(4))
    assert np.allclose(s, np.sort(np.abs(d))[::-1], rtol=8 * EPS64, atol=1e-18 * 7.5)
    assert np.all(_gpu_sigma(bb, np.zeros(6), np.zeros(5)) == 0.0)
    n = 300
    d = 10.0 ** (-6.0 * np.arange(n) / n)
    e = 0.5 * 10.0 ** (-6.0 * np.arange(1, n) / n)
    _check_sigma(bb, d, e)
    a, b, c = 3.0, 4.0, 2.0        # B = [[a, b], [0, c]]
    fro2, det = a * a + b * b + c * c, abs(a * c)
    smax = np.sqrt((fro2 + np.sqrt(fro2 * fro2 - 4 * det * det)) / 2)
    s = _gpu_sigma(bb, np.array([a, c]), np.array([b]))
    assert abs(s[0] - smax) <= 8 * EPS64 * smax and abs(s[1] - det / smax) <= 8 * EPS64 * smax


def test_bidiag_sigma_power_of_two_scaling_is_exact(bb):
    """The count runs on the matrix scaled by a power of two (max |b| in [1/2, 1)),
    so sigma(2^k B) is 2^k sigma(B) bit for bit, also where the squares of the
    unscaled entries would overflow (k = 600, 1000) or underflow (k = -600, -1000)."""
    _say("case bidiag sigma 2^k scaling")
    rng = np.random.default_rng(11)
    n = 777
    d = 2.0 + np.abs(rng.standard_normal(n))     # well conditioned: no sigma near the underflow range
    e = 0.5 * rng.standard_normal(n - 1)
    s0 = _gpu_sigma(bb, d, e)
    _check_sigma(bb, d, e)
    for k in (600, -600, 1000, -1000):
        s = _gpu_sigma(bb, np.ldexp(d, k), np.ldexp(e, k))
        assert np.array_equal(s, np.ldexp(s0, k)), k


def test_bidiag_sigma_graded_diagonal_relative_accuracy(bb):
    """A diagonal B whose entries fall from 2 to 2^-8 (the range in which the stop
    at 4 eps of the interval's upper end, not the 2^-60 ||B|| floor, decides):
    every sigma is some |d_i|, found to a few ulps of itself."""
    _say("case bidiag sigma graded diagonal")
    n = 500
    rng = np.random.default_rng(12)
    d = np.ldexp(1.0 + rng.random(n), -(np.arange(n) * 9) // n) * np.where(rng.random(n) < 0.5, -1.0, 1.0)
    s = _gpu_sigma(bb, d, np.zeros(n - 1))
    ref = np.sort(np.abs(d))[::-1]
    assert np.all(np.abs(s - ref) <= 8 * EPS64 * ref), np.max(np.abs(s - ref) / ref)


def test_bidiag_sigma_non_finite_input_gives_nan(bb):
    _say("case bidiag sigma non-finite input")
    d = np.ones(10)
    e = np.full(9, 0.5)
    for bad in (np.nan, np.inf, -np.inf):
        d2 = d.copy()
        d2[3] = bad
        assert np.all(np.isnan(_gpu_sigma(bb, d2, e)))
        e2 = e.copy()
        e2[8] = bad
        assert np.all(np.isnan(_gpu_sigma(bb, d, e2)))


def test_bidiag_sigma_after_reduction(bb):
    """The full second + third stage on the device: reduce the n = 8192, b = 64 band,
    then sigma of the result, against the oracle's sigma of the same (d, e) and, through
    the bitwise reduction parity, of the oracle's own bidiagonal."""
    n, b = 8192, 64
    _say("case reduction + device sigma n=8192 b=64")
    band = inputs.workload("n8192_b64")
    t = torch.from_numpy(band).cuda()
    d, e = bb.bb_reduce(t, n, b)
    s = bb.bidiag_sigma(d, e)
    torch.cuda.synchronize()
    s = s.cpu().numpy()
    s_ref = oracle.singular_values(d.cpu().numpy(), e.cpu().numpy())
    assert np.max(np.abs(s - s_ref)) <= 20 * n * EPS64 * s_ref[0]
    A2 = np.sum(band * band)
    assert abs(np.sum(s * s) - A2) <= 40 * n * EPS64 * A2


# ------------------------------------------------------------------ ragged batch
def _batch_case(count, seed, n_lo, n_hi, bands):
    return inputs.ragged_batch(count=count, seed=seed, n_lo=n_lo, n_hi=n_hi, bands=bands)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_batched_equals_individual_calls_bitwise(bb, dtype):
    """One persistent launch over a ragged batch computes exactly what one
    bb_reduce per matrix computes (same per-task arithmetic, same order)."""
    _say("case ragged batch of 24, %s" % dtype)
    mats = _batch_case(24, 7, 40, 700, (3, 16, 33))
    mats.append((1, 4, np.array([[0.0, 0.0, 0.0, 0.0, 1.5]])))   # n = 1
    mats.append((2, 1, np.array([[0.0, 1.0], [2.0, 3.0]])))      # bidiagonal already
    bb.reset_params()
    bb.set_params(tw=16 if dtype == torch.float64 else 32)
    bands = [torch.from_numpy(np.ascontiguousarray(bd)).cuda().to(dtype) for (_, _, bd) in mats]
    ns = [m[0] for m in mats]
    bs = [m[1] for m in mats]
    ds, es = bb.bb_reduce_batched(bands, ns, bs)
    assert bb.stream_status() == 0
    for t, n, b, dd, ee in zip(bands, ns, bs, ds, es):
        d1, e1 = bb.bb_reduce(t, n, b)
        assert np.array_equal(dd.cpu().numpy(), d1.cpu().numpy())
        assert np.array_equal(ee.cpu().numpy(), e1.cpu().numpy())
    # FP64: also the oracle, bitwise
    if dtype == torch.float64:
        for (n, b, bd), dd, ee in list(zip(mats, ds, es))[:6]:
            do, eo = oracle.reduce(bd, n, b, 16)
            assert np.array_equal(dd.cpu().numpy(), do) and np.array_equal(ee.cpu().numpy(), eo)
    bb.reset_params()


def test_batched_fp16_matches_individual_calls(bb):
    mats = _batch_case(12, 9, 64, 400, (16, 32))
    bb.reset_params()
    bands = [torch.from_numpy(bd).cuda().to(torch.float16) for (_, _, bd) in mats]
    ns = [m[0] for m in mats]
    bs = [m[1] for m in mats]
    ds, es = bb.bb_reduce_batched(bands, ns, bs)
    for t, n, b, dd, ee in zip(bands, ns, bs, ds, es):
        d1, e1 = bb.bb_reduce(t, n, b)
        assert np.array_equal(dd.cpu().numpy(), d1.cpu().numpy())
        assert np.array_equal(ee.cpu().numpy(), e1.cpu().numpy())


def test_batched_graph_capture_replays(bb):
    """The batched call captured into a hipGraph replays correctly several times,
    with eager work and synchronisation between the replays."""
    mats = _batch_case(16, 11, 64, 500, (16, 32, 64))
    bb.reset_params()
    bands = [torch.from_numpy(bd).cuda().to(torch.float32) for (_, _, bd) in mats]
    ns = [m[0] for m in mats]
    bs = [m[1] for m in mats]
    ds = [torch.empty(max(n, 1), dtype=torch.float64, device="cuda") for n in ns]
    es = [torch.empty(max(n - 1, 1), dtype=torch.float64, device="cuda") for n in ns]
    ref_d, ref_e = bb.bb_reduce_batched(bands, ns, bs, ds=ds, es=es)   # eager call builds the plan
    ref_d = [x.cpu().numpy().copy() for x in ref_d]
    ref_e = [x.cpu().numpy().copy() for x in ref_e]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        bb.bb_reduce_batched(bands, ns, bs, ds=ds, es=es, stream=s)     # warm the plan on this stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        bb.bb_reduce_batched(bands, ns, bs, ds=ds, es=es, stream=s)
    for rep in range(3):
        for x in ds:
            x.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for x, rd in zip(ds, ref_d):
            assert np.array_equal(x[: len(rd)].cpu().numpy(), rd)
        for x, re_ in zip(es, ref_e):
            assert np.array_equal(x[: len(re_)].cpu().numpy(), re_)
        _ = torch.ones(1000, device="cuda").sum().item()   # eager work between replays


_WATCHDOG_CHILD = r"""
import sys
sys.path.insert(0, sys.argv[1])
import numpy as np, torch
from paper_2510_12705_amd import bb, inputs
n, b = 4096, 64
band = torch.from_numpy(inputs.band_normal(n, b, seed=11)).cuda()
d = torch.empty(n, dtype=torch.float64, device="cuda")
e = torch.empty(n, dtype=torch.float64, device="cuda")
rc = bb.lib.bb_reduce(n, b, bb.F64, band.data_ptr(), b + 1, d.data_ptr(), e.data_ptr(), None)
st = bb.lib.bb_stream_status(None)
print("RESULT", rc, st, flush=True)
"""


def test_watchdog_turns_stalled_waits_into_timeout_error(tmp_path):
    """A spin limit of one makes every dependency wait give up after its first check:
    the pipeline must drain (every workgroup exits through the abort word) and the
    call must report BB_ERR_TIMEOUT (or success if no wait lasted that long)."""
    import os
    import subprocess
    import sys
    _say("case watchdog with BB_SPIN_LIMIT=1")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    script = tmp_path / "child.py"
    script.write_text(_WATCHDOG_CHILD)
    env = dict(os.environ, BB_SPIN_LIMIT="1")
    r = subprocess.run([sys.executable, str(script), root], env=env, capture_output=True, text=True, timeout=110)
    assert r.returncode == 0, r.stderr[-2000:]
    line = [x for x in r.stdout.splitlines() if x.startswith("RESULT")][-1]
    _, rc, st = line.split()
    assert int(rc) == 0
    assert int(st) in (0, 2), st
