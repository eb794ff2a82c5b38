"""Pins of the accuracy experiment's input recipe (Sec. V-A): prescribed spectra
in [0, 1], Haar orthogonal factors, and the FP64 block Householder reduction of
U diag(sigma) V^T to an upper band that keeps sigma."""
import math

import numpy as np
import pytest

from paper_2510_12705_amd import accuracy as acc
from tests.pins import band_to_dense


def test_spectra_shapes():
    rng = np.random.default_rng(0)
    s = acc.spectrum("arithmetic", 8, rng)
    assert np.array_equal(s, np.array([8, 7, 6, 5, 4, 3, 2, 1]) / 8.0)
    s = acc.spectrum("logarithmic", 7, rng)
    assert s[0] == 1.0 and abs(s[-1] - 1e-6) < 1e-20 and np.all(np.diff(np.log10(s)) == pytest.approx(-1.0))
    s = acc.spectrum("quarter-circle", 200000, np.random.default_rng(1))
    assert np.all(np.diff(s) <= 0) and s.min() >= 0.0 and s.max() <= 1.0
    # moments of the quarter-circle law on [0, 1] (density (4/pi) sqrt(1 - x^2)): E x = 4 / (3 pi), E x^2 = 1/4
    assert abs(s.mean() - 4.0 / (3.0 * math.pi)) < 5e-3
    assert abs(np.mean(s * s) - 0.25) < 5e-3


def test_haar_factor_is_orthogonal():
    Q = acc.haar_orthogonal(50, np.random.default_rng(3))
    assert np.abs(Q.T @ Q - np.eye(50)).max() < 1e-13


@pytest.mark.parametrize("n,b", [(120, 7), (64, 63), (90, 1), (33, 32), (100, 40)])
@pytest.mark.parametrize("kind", acc.SPECTRA)
def test_dense_to_band_keeps_the_spectrum(n, b, kind):
    band, s = acc.test_matrix(kind, n, b, seed=n + b)
    A = band_to_dense(band, n, b)
    # the band array holds nothing outside the band (A(i, j) = 0 unless 0 <= j - i <= b)
    for j in range(min(b, n)):
        assert np.all(band[j, : b - j] == 0.0)
    sv = np.linalg.svd(A, compute_uv=False)
    assert np.max(np.abs(sv - s)) <= 50 * n * np.finfo(float).eps * s[0]


def test_dense_to_band_is_the_identity_on_a_band_up_to_signs():
    # a matrix that is already upper triangular with b super-diagonals keeps its band
    # structure (each panel QR / LQ acts on an already reduced panel)
    n, b = 40, 5
    rng = np.random.default_rng(7)
    A = np.triu(rng.standard_normal((n, n))) - np.triu(rng.standard_normal((n, n)), b + 1) * 0.0
    A = np.triu(A) * (np.abs(np.subtract.outer(np.arange(n), np.arange(n))) <= b)
    band = acc.dense_to_band(A, b)
    B = band_to_dense(band, n, b)
    assert np.allclose(np.abs(B), np.abs(A), atol=1e-12)
