"""Pins of the CPU oracle against facts fixed by the mathematics (CPU only).

Each test targets a different class of plausible mistake:
  * index ranges / storage      -> dense full-range coding equals the band oracle exactly
  * arithmetic of reflectors    -> singular values vs brute-force Jacobi, Frobenius norm
  * sign / transposed operands  -> U^T A V = B with orthogonal U, V
  * Householder convention      -> closed forms d0 = a00, |e0| = ||A[0,1:]||, n = 3 formula
  * zero handling (tau = 0)     -> already-bidiagonal input returned bitwise unchanged
  * uniqueness (implicit Q)     -> |d|,|e| equal a textbook dense Golub-Kahan bidiagonalisation
"""
import math

import numpy as np
import pytest

import oracle
from paper_2510_12705_amd import inputs
from tests.pins import band_to_dense, dense_to_band, golub_kahan_dense, jacobi_singular_values

EPS = np.finfo(np.float64).eps


def _bidiag(d, e):
    n = len(d)
    B = np.diag(d)
    if n > 1:
        B += np.diag(e, 1)
    return B


CASES = [(12, 3, 1), (12, 3, 2), (20, 5, 2), (24, 6, 2), (24, 6, 4), (31, 7, 3), (17, 16, 16),
         (25, 8, 7), (30, 9, 1), (16, 4, 16), (9, 8, 3), (40, 12, 5)]


@pytest.mark.parametrize("n,b,tw", CASES)
def test_band_equals_dense_full_range(n, b, tw):
    """Band oracle (exact application ranges) == pure-Python dense chase that applies every
    reflector to every row and column; the dense result is exactly bidiagonal."""
    band = inputs.band_normal(n, b, seed=100 + n + b + tw)
    A = band_to_dense(band, n, b)
    M = np.array(oracle.reduce_dense_full(A.tolist(), b, tw))
    off = M - np.diag(np.diag(M)) - np.diag(np.diag(M, 1), 1)
    assert np.count_nonzero(off) == 0, "dense full-range chase left off-bidiagonal entries"
    d, e = oracle.reduce(band, n, b, tw)
    assert np.array_equal(d, np.diag(M))
    assert np.array_equal(e, np.diag(M, 1))


@pytest.mark.parametrize("n,b,tw", [(40, 6, 2), (64, 10, 3), (48, 16, 16), (33, 32, 8)])
def test_singular_values_vs_jacobi(n, b, tw):
    band = inputs.band_normal(n, b, seed=7 + n)
    A = band_to_dense(band, n, b)
    d, e = oracle.reduce(band, n, b, tw)
    s = oracle.singular_values(d, e)
    sj = jacobi_singular_values(A)
    assert np.max(np.abs(s - sj)) <= 4 * n * EPS * sj[0]
    # library cross-check of the same dense matrix
    sl = np.linalg.svd(A, compute_uv=False)
    assert np.max(np.abs(s - sl)) <= 4 * n * EPS * sl[0]


def test_singular_values_routine_vs_dense_svd():
    """The TGK/dsterf routine applied to a bidiagonal equals a dense SVD of that bidiagonal."""
    rng = np.random.default_rng(3)
    d, e = rng.standard_normal(50), rng.standard_normal(49)
    s = oracle.singular_values(d, e)
    sl = np.linalg.svd(_bidiag(d, e), compute_uv=False)
    assert np.max(np.abs(s - sl)) <= 10 * 50 * EPS * sl[0]


@pytest.mark.parametrize("n,b,tw", [(64, 8, 3), (100, 16, 16), (96, 24, 5)])
def test_frobenius_preserved(n, b, tw):
    band = inputs.band_uniform(n, b, seed=11)
    A = band_to_dense(band, n, b)
    d, e = oracle.reduce(band, n, b, tw)
    lhs = np.sum(d * d) + np.sum(e * e)
    rhs = np.sum(A * A)
    assert abs(lhs - rhs) <= 10 * n * EPS * rhs


@pytest.mark.parametrize("n,b,tw", [(30, 5, 2), (48, 9, 4), (40, 12, 11)])
def test_orthogonal_factors(n, b, tw):
    band = inputs.band_normal(n, b, seed=21)
    A = band_to_dense(band, n, b)
    d, e, U, V = oracle.reduce(band, n, b, tw, want_uv=True)
    I = np.eye(n)
    assert np.linalg.norm(U.T @ U - I) <= 10 * n * EPS
    assert np.linalg.norm(V.T @ V - I) <= 10 * n * EPS
    B = _bidiag(d, e)
    assert np.linalg.norm(U.T @ A @ V - B) <= 10 * n * EPS * np.linalg.norm(A)
    # no reflector ever touches row 0 / column 0 from the left, or column 0 from the right
    assert np.array_equal(U[:, 0], I[:, 0])
    assert np.array_equal(V[:, 0], I[:, 0])


@pytest.mark.parametrize("n,b,tw", [(50, 7, 3), (64, 32, 16), (20, 19, 4)])
def test_closed_forms_first_row(n, b, tw):
    band = inputs.band_normal(n, b, seed=31)
    A = band_to_dense(band, n, b)
    d, e = oracle.reduce(band, n, b, tw)
    assert d[0] == A[0, 0]
    assert abs(abs(e[0]) - np.linalg.norm(A[0, 1:])) <= 4 * EPS * np.linalg.norm(A[0, 1:])


def test_n3_closed_form():
    """n = 3, b = 2: one right reflector on columns 1..2 of row 0 and one left reflector.
    With u = (a01, a02)/||(a01, a02)|| and M the trailing 2x2 block: |d1| = ||M u||,
    |d1 d2| = |a11 a22|, and d1^2 + e1^2 + d2^2 = ||M||_F^2."""
    for seed in range(5):
        rng = np.random.default_rng(seed)
        a = rng.standard_normal(6)
        A = np.array([[a[0], a[1], a[2]], [0, a[3], a[4]], [0, 0, a[5]]])
        band = dense_to_band(A, 2)
        d, e = oracle.reduce(band, 3, 2, 1)
        u = A[0, 1:] / np.linalg.norm(A[0, 1:])
        M = A[1:, 1:]
        d1 = np.linalg.norm(M @ u)
        d2 = abs(a[3] * a[5]) / d1
        e1 = math.sqrt(max(np.sum(M * M) - d1 * d1 - d2 * d2, 0.0))
        assert d[0] == a[0]
        assert abs(abs(e[0]) - np.linalg.norm(A[0, 1:])) <= 4 * EPS * np.linalg.norm(A[0, 1:])
        assert abs(abs(d[1]) - d1) <= 16 * EPS * d1
        assert abs(abs(d[2]) - d2) <= 16 * EPS * max(d2, 1e-300)
        assert abs(abs(e[1]) - e1) <= 1e-7 * np.linalg.norm(M)


@pytest.mark.parametrize("n,b,tw", [(30, 6, 2), (25, 8, 3), (40, 5, 4)])
def test_bidiagonal_input_unchanged(n, b, tw):
    rng = np.random.default_rng(5)
    A = np.diag(rng.standard_normal(n)) + np.diag(rng.standard_normal(n - 1), 1)
    band = dense_to_band(A, b)
    d, e = oracle.reduce(band, n, b, tw)
    assert np.array_equal(d, np.diag(A))
    assert np.array_equal(e, np.diag(A, 1))


def test_degenerate_sizes():
    # n = 0
    d, e = oracle.reduce(np.zeros((0, 4)), 0, 3, 2)
    assert d.size == 0 and e.size == 0
    # n = 1
    d, e = oracle.reduce(np.array([[0.0, 0.0, 2.5]]), 1, 2, 1)
    assert d.tolist() == [2.5] and e.size == 0
    # b = 0: diagonal passes through
    band = np.arange(1.0, 6.0).reshape(5, 1)
    d, e = oracle.reduce(band, 5, 0, 4)
    assert d.tolist() == [1, 2, 3, 4, 5] and e.tolist() == [0, 0, 0, 0]
    # n = 2 with b = 1: already bidiagonal
    band = np.array([[0.0, 1.0], [2.0, 3.0]])
    d, e = oracle.reduce(band, 2, 1, 4)
    assert d.tolist() == [1.0, 3.0] and e.tolist() == [2.0]
    # b >= n is clamped to n - 1
    n = 6
    band = inputs.band_normal(n, 9, seed=1)
    A = band_to_dense(band, n, 9)
    d, e = oracle.reduce(band, n, 9, 2)
    s = oracle.singular_values(d, e)
    assert np.allclose(s, np.linalg.svd(A, compute_uv=False), atol=1e-13)


def test_invalid_arguments():
    with pytest.raises(ValueError):
        oracle.reduce(np.zeros((4, 3)), 4, 2, 0)       # TW < 1
    with pytest.raises(ValueError):
        oracle.reduce(np.zeros((4, 2)), 4, 2, 1)       # ldband < b+1


def _well_conditioned_band(n, b, seed):
    band = inputs.band_normal(n, b, seed)
    band[:, b] += 3.0 * math.sqrt(b + 1)   # dominant diagonal keeps B far from splitting
    return band


@pytest.mark.parametrize("n,b", [(40, 6), (64, 12), (80, 20)])
def test_unique_up_to_sign_vs_golub_kahan(n, b):
    band = _well_conditioned_band(n, b, seed=41)
    A = band_to_dense(band, n, b)
    dg, eg = golub_kahan_dense(A)
    for tw in sorted({1, 2, 3, b - 1}):
        d, e = oracle.reduce(band, n, b, tw)
        nrm = np.linalg.norm(A)
        assert np.max(np.abs(np.abs(d) - np.abs(dg))) <= 1e-12 * nrm
        assert np.max(np.abs(np.abs(e) - np.abs(eg))) <= 1e-12 * nrm


@pytest.mark.parametrize("n,b,tw", [(40, 8, 2), (45, 10, 4), (33, 6, 5), (50, 16, 16), (29, 5, 3)])
def test_pipelined_order_is_bitwise_sequential(n, b, tw):
    """Random interleavings allowed by the half-step lag rule H = (4, 3, 2) for
    c = (1, 2, >=3) reproduce the sequential oracle bitwise."""
    band = inputs.band_normal(n, b, seed=n * b)
    d0, e0 = oracle.reduce(band, n, b, tw)
    for seed in range(1, 9):
        d, e = oracle.reduce_pipelined(band, n, b, tw, (4, 3, 2), seed)
        assert np.array_equal(d, d0) and np.array_equal(e, e0)


@pytest.mark.parametrize("n,b,tw,threads,group", [(40, 8, 2, 4, 1), (300, 17, 4, 8, 1), (257, 33, 16, 3, 3),
                                                  (200, 64, 32, 8, 8), (64, 5, 1, 8, 2), (300, 9, 4, 8, 5),
                                                  (100, 3, 1, 4, 256), (3, 2, 1, 2, 1), (1, 4, 4, 2, 4)])
def test_wavefront_threads_are_bitwise_sequential(n, b, tw, threads, group):
    """The multi-threaded wavefront (the CPU timing baseline) runs the same
    half-steps under the lag rule on real threads, one sweep or a group of
    sweeps per thread at a time: bitwise the sequential oracle."""
    band = inputs.band_normal(n, b, seed=n + b)
    d0, e0 = oracle.reduce(band, n, b, tw)
    for _ in range(3):
        d, e, used = oracle.reduce_wavefront(band, n, b, tw, threads=threads, group=group)
        assert used == (threads if b > 1 and n > 2 else 1)   # no stage runs: no team
        assert np.array_equal(d, d0) and np.array_equal(e, e0)


def test_wavefront_stage_limit_matches_a_one_stage_reduction():
    """With b = tw + 1 the first stage is the whole reduction, so a one-stage
    sample must equal the full sequential result; with two stages it must not
    reach it (the sample really stops)."""
    n, b, tw = 120, 9, 8
    band = inputs.band_normal(n, b, seed=4)
    d0, e0 = oracle.reduce(band, n, b, tw)
    d, e, _ = oracle.reduce_wavefront(band, n, b, tw, threads=4, group=2, max_stages=1)
    assert np.array_equal(d, d0) and np.array_equal(e, e0)
    d0, e0 = oracle.reduce(band, n, b, 4)   # 9 -> 5 -> 1
    d, e, _ = oracle.reduce_wavefront(band, n, b, 4, threads=4, group=2, max_stages=1)
    assert not np.array_equal(e, e0)
    d, e, _ = oracle.reduce_wavefront(band, n, b, 4, threads=4, group=2, max_stages=2)
    assert np.array_equal(d, d0) and np.array_equal(e, e0)


def test_pipelined_detects_unsafe_rule():
    """Planted mistake: a lag one half-step too short must change the result for some order."""
    n, b, tw = 40, 8, 2   # c = 6 >= 3, safe lag 2, unsafe lag 1
    band = inputs.band_normal(n, b, seed=9)
    d0, e0 = oracle.reduce(band, n, b, tw)
    differs = False
    for seed in range(1, 30):
        d, e = oracle.reduce_pipelined(band, n, b, tw, (4, 3, 1), seed)
        if not (np.array_equal(d, d0) and np.array_equal(e, e0)):
            differs = True
            break
    assert differs


@pytest.mark.parametrize("n,b,tw", [(30, 6, 2), (40, 9, 4)])
def test_power_of_two_scaling_is_exact(n, b, tw):
    """Scaling A by 2^-1000 pushes every reflector into the |beta| < safmin rescaling
    branch; a power-of-two scale commutes exactly with every operation, so d and e
    must scale exactly (a missing scale-back of beta, or an overflowing 1/(alpha-beta),
    breaks this).  A diagonally dominant band keeps every intermediate value normal."""
    band = _well_conditioned_band(n, b, seed=77)
    d0, e0 = oracle.reduce(band, n, b, tw)
    s = 2.0 ** -1000
    d1, e1 = oracle.reduce(band * s, n, b, tw)
    assert np.isfinite(d1).all() and np.isfinite(e1).all()
    assert np.array_equal(d1, d0 * s) and np.array_equal(e1, e0 * s)
    A = band_to_dense(band * s, n, b)
    M = np.array(oracle.reduce_dense_full(A.tolist(), b, tw))
    assert np.array_equal(d1, np.diag(M)) and np.array_equal(e1, np.diag(M, 1))


def test_long_band_stays_finite():
    """N(0,1) triangular bands are exponentially ill-conditioned: at n = 4096 the
    super-diagonal underflows; every output must still be finite."""
    n, b = 4096, 64
    band = inputs.band_normal(n, b, seed=1)
    d, e = oracle.reduce(band, n, b, 16)
    assert np.isfinite(d).all() and np.isfinite(e).all()
    A2 = np.sum(band * band)
    assert abs(np.sum(d * d) + np.sum(e * e) - A2) <= 100 * n * EPS * A2


@pytest.mark.parametrize("scale", [1.0, 1e-300, 1e300, 2.0 ** -540, 2.0 ** 500])
def test_nrm2_safe_scaling_matches_definition(scale):
    """The norm used by the reflector generator (LAPACK >= 3.10 xNRM2) equals the
    Euclidean norm within a few ulps in every magnitude regime, including mixed
    tiny / mid / huge entries that go to different accumulators."""
    rng = np.random.default_rng(1)
    x = rng.standard_normal(33) * scale
    exact = float(np.sqrt(np.sum((x / scale) ** 2))) * scale
    assert abs(oracle._nrm2(x.tolist()) - exact) <= 8 * EPS * exact
    mixed = [1e-310, 3.0, 1e-200, 4.0] if scale == 1.0 else [scale, 1e-320, 2.0 * scale]
    ref = math.sqrt(sum((v / max(mixed)) ** 2 for v in mixed)) * max(mixed)
    assert abs(oracle._nrm2(mixed) - ref) <= 8 * EPS * ref


_NRM2_CASES = [
    [3.0, 4.0],                                   # mid range only
    [2.0 ** 600, 2.0 ** 600, -(2.0 ** 601)],      # huge only (abig accumulator)
    [2.0 ** 487, 2.0 ** 486],                     # huge + mid at the tbig threshold
    [2.0 ** 700, 1.0, -3.0, 2.0 ** 699],          # huge + mid combined
    [2.0 ** 700, 1e-300, 5e-324],                 # huge + tiny (tiny ignored)
    [1e-300, -2e-300, 3e-310],                    # tiny only (asml accumulator)
    [1e-300, 3.0, 1e-200, 4.0],                   # tiny + mid combined
    [2.0 ** -511, 2.0 ** -512],                   # tiny / mid threshold
    [0.0, 0.0, 2.0 ** 1000, 0.0],                 # zeros and one huge value
    [1.0e308, -1.0e308],                          # overflows as a plain sum of squares
]


@pytest.mark.parametrize("x", _NRM2_CASES)
def test_c_nrm2_every_regime(x):
    """The C oracle's xNRM2 itself (not only its Python twin): the Euclidean norm
    within 2 ulp (Python's math.hypot of many arguments is the reference) in every
    accumulator regime, and bitwise equal to the independent Python coding."""
    ref = math.hypot(*x)
    got = oracle.nrm2(np.array(x))
    assert abs(got - ref) <= 2 * EPS * ref, (got, ref)
    assert got == oracle._nrm2(x)


@pytest.mark.parametrize("n,b,tw", [(30, 6, 2), (40, 9, 4), (24, 12, 11)])
def test_huge_scaling_takes_the_big_accumulator_exactly(n, b, tw):
    """Scaling A by 2^600 puts every nonzero entry above xNRM2's 2^486 threshold, so
    every norm goes through the huge-value accumulator (scaled by 2^-538) of the C
    oracle.  A power of two commutes with each operation, so d and e must scale
    exactly, and the band oracle must equal the dense full-range chase (whose norm is
    the separate Python coding) bit for bit."""
    band = _well_conditioned_band(n, b, seed=78)
    d0, e0 = oracle.reduce(band, n, b, tw)
    s = 2.0 ** 600
    d1, e1 = oracle.reduce(band * s, n, b, tw)
    assert np.isfinite(d1).all() and np.isfinite(e1).all()
    assert np.array_equal(d1, d0 * s) and np.array_equal(e1, e0 * s)
    A = band_to_dense(band * s, n, b)
    M = np.array(oracle.reduce_dense_full(A.tolist(), b, tw))
    assert np.array_equal(d1, np.diag(M)) and np.array_equal(e1, np.diag(M, 1))
