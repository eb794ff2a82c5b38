"""Singular-vector path (bb_reduce_vectors): U^T A V = bidiag(d, e).

Against the oracle, which accumulates U <- U H and V <- V H for every reflector
in the sequential order of the reduction (the same definition, run on the CPU):
  * FP64 storage: d, e bitwise those of bb_reduce, U and V equal to the
    oracle's (np.array_equal: bitwise up to the sign of zero);
  * every storage type: ||U^T U - I||, ||V^T V - I|| <= 20 n eps64 (the logged
    reflectors are FP64), U e1 = V e1 = e1 exactly, and ||U^T A V - B||_F within
    a multiple of n eps ||A||_F for the storage type's eps;
  * only one of U, V asked for; tiny and degenerate shapes; a 64-wide tile.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2510_12705_amd import inputs  # noqa: E402
from tests.pins import band_to_dense  # noqa: E402

EPS = {torch.float64: np.finfo(np.float64).eps, torch.float32: np.finfo(np.float32).eps,
       torch.float16: np.finfo(np.float16).eps}


@pytest.fixture(scope="module")
def bb():
    from paper_2510_12705_amd import bb as _bb
    _bb.reset_params()
    yield _bb
    _bb.reset_params()


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _vectors(bb, band, n, b, dt, **params):
    bb.reset_params()
    if params:
        bb.set_params(**params)
    t = torch.from_numpy(np.ascontiguousarray(band)).to("cuda:0").to(dt)
    d, e, U, V = bb.bb_reduce_vectors(t, n, b)
    d1, e1 = bb.bb_reduce(t, n, b)
    st = bb.stream_status()
    tw = bb.resolved_params(n, b, bb._torch_dtype_code(t)).tw
    bb.reset_params()
    assert st == 0, bb.bb_error_string(st)
    d, e = d.cpu().numpy(), e.cpu().numpy()
    assert np.array_equal(d, d1.cpu().numpy()) and np.array_equal(e, e1.cpu().numpy())
    return d, e, U.cpu().numpy(), V.cpu().numpy(), tw


def _bidiag(d, e):
    n = len(d)
    B = np.diag(d)
    if n > 1:
        B += np.diag(e, 1)
    return B


def _check_factors(band, n, b, d, e, U, V, eps, k):
    A = band_to_dense(band, n, b)
    I = np.eye(n)
    e64 = np.finfo(np.float64).eps
    assert np.abs(U.T @ U - I).max() <= 20 * n * e64
    assert np.abs(V.T @ V - I).max() <= 20 * n * e64
    assert np.array_equal(U[:, 0], I[:, 0]) and np.array_equal(V[:, 0], I[:, 0])
    R = U.T @ A @ V - _bidiag(d, e)
    nA = np.linalg.norm(A)
    err = np.linalg.norm(R) / nA
    _say("  ||U^T A V - B||_F / ||A||_F = %.3e (%.3f n eps)" % (err, err / (n * eps)))
    assert err <= k * n * eps


@pytest.mark.parametrize("n,b,tw", [(300, 17, 4), (513, 40, 32), (700, 64, 16), (1024, 9, 8), (257, 3, 1)])
def test_fp64_factors_equal_the_oracles(bb, n, b, tw):
    _say("case vectors fp64 n=%d b=%d tw=%d" % (n, b, tw))
    band = inputs.band_normal(n, b, seed=n + 3 * b)
    d, e, U, V, twu = _vectors(bb, band, n, b, torch.float64, tw=tw)
    assert twu == tw
    do, eo, Uo, Vo = oracle.reduce(band, n, b, tw, want_uv=True)
    assert np.array_equal(d, do) and np.array_equal(e, eo)
    assert np.array_equal(U, Uo), np.flatnonzero(U != Uo)[:5]
    assert np.array_equal(V, Vo), np.flatnonzero(V != Vo)[:5]
    _check_factors(band, n, b, d, e, U, V, EPS[torch.float64], 20)


def test_fp64_default_launch_n2048(bb):
    n, b = 2048, 64
    _say("case vectors fp64 n=%d b=%d default launch" % (n, b))
    band = inputs.band_normal(n, b, seed=2)
    d, e, U, V, tw = _vectors(bb, band, n, b, torch.float64)
    do, eo, Uo, Vo = oracle.reduce(band, n, b, tw, want_uv=True)
    assert np.array_equal(U, Uo) and np.array_equal(V, Vo)
    _check_factors(band, n, b, d, e, U, V, EPS[torch.float64], 20)


@pytest.mark.parametrize("dt,n,b,params", [(torch.float32, 1500, 64, {}), (torch.float32, 900, 130, {"tw": 64}),
                                           (torch.float16, 800, 48, {})])
def test_reduced_precision_factors(bb, dt, n, b, params):
    _say("case vectors %s n=%d b=%d %r" % (dt, n, b, params))
    band = inputs.band_uniform(n, b, seed=n + b)
    rb = band.astype({torch.float32: np.float32, torch.float16: np.float16}[dt]).astype(np.float64)
    d, e, U, V, _ = _vectors(bb, rb, n, b, dt, **params)
    _check_factors(rb, n, b, d, e, U, V, EPS[dt], 20 if dt == torch.float32 else 2)


def test_one_factor_only_and_small_shapes(bb):
    n, b = 400, 20
    band = inputs.band_normal(n, b, seed=8)
    t = torch.from_numpy(band).cuda()
    _, _, U, Vnone = bb.bb_reduce_vectors(t, n, b, want_v=False)
    _, _, Unone, V = bb.bb_reduce_vectors(t, n, b, want_u=False)
    assert Vnone is None and Unone is None
    _, _, U2, V2 = bb.bb_reduce_vectors(t, n, b)
    assert bb.stream_status() == 0
    assert np.array_equal(U.cpu().numpy(), U2.cpu().numpy()) and np.array_equal(V.cpu().numpy(), V2.cpu().numpy())
    for (n, b) in [(1, 0), (2, 1), (3, 2), (5, 0), (6, 1), (7, 10), (40, 39)]:
        band = inputs.band_normal(n, b, seed=n)
        t = torch.from_numpy(band).cuda()
        d, e, U, V = bb.bb_reduce_vectors(t, n, b)
        assert bb.stream_status() == 0
        d, e, U, V = d.cpu().numpy(), e.cpu().numpy(), U.cpu().numpy(), V.cpu().numpy()
        bq = min(b, n - 1)
        tw = bb.resolved_params(n, b, bb.F64).tw
        do, eo, Uo, Vo = oracle.reduce(band, n, b, tw, want_uv=True)
        assert np.array_equal(d, do) and np.array_equal(e, eo), (n, b)
        assert np.array_equal(U, Uo) and np.array_equal(V, Vo), (n, b, bq)


def test_factors_on_a_side_stream_are_complete_when_that_stream_is(bb):
    """The accumulation runs on a second, library-owned stream beside the reduction
    and is joined back into the caller's stream: on a non-default stream, waiting
    for that stream alone must give the factors of a default-stream call, bitwise,
    also when the caller reuses the output buffers right away."""
    n, b = 1500, 48
    _say("case vectors side stream n=%d b=%d" % (n, b))
    band = inputs.band_normal(n, b, seed=11)
    t = torch.from_numpy(np.ascontiguousarray(band)).to("cuda:0")
    bb.reset_params()
    d0, e0, U0, V0 = bb.bb_reduce_vectors(t, n, b)
    torch.cuda.synchronize()
    ref = [x.cpu().numpy() for x in (d0, e0, U0, V0)]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        d, e, U, V = bb.bb_reduce_vectors(t, n, b, stream=s)
        Uc, Vc = U.clone(), V.clone()   # queued on s right behind the call
        U.zero_()
        V.zero_()
    s.synchronize()
    assert bb.stream_status(s) == 0
    got = [x.cpu().numpy() for x in (d, e, Uc, Vc)]
    for a, r in zip(got, ref):
        assert np.array_equal(a, r)
