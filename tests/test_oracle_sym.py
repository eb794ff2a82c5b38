"""Pins of the symmetric oracle (band -> tridiagonal, A <- H A H per step).

What fixes it independently of its own code:
  * eigenvalues equal numpy's eigvalsh of the dense symmetric matrix;
  * Q^T A Q = tridiag(d, e) with the accumulated Q orthogonal and Q e1 = e1;
  * by the implicit-Q theorem the tridiagonal with Q e1 = e1 is unique up to
    signs: |d|, |e| equal those of LAPACK's Householder Hessenberg reduction
    (scipy.linalg.hessenberg, which also fixes e1) of the dense matrix;
  * closed forms: d0 = a00 bitwise, |e0| = ||A[1:b+1, 0]||, Frobenius norm;
  * a tridiagonal input comes back bitwise; b = 0 and n <= 2 degenerate cases.
"""
import numpy as np
import pytest
import scipy.linalg

import oracle

EPS = np.finfo(np.float64).eps


def sym_band(n, b, seed, dominant=False):
    rng = np.random.default_rng(seed)
    band = rng.standard_normal((n, b + 1))
    if dominant:
        band[:, 0] += 4.0 * (b + 1)
    for j in range(n):      # entries below row n-1 do not exist
        band[j, max(0, n - j):] = 0.0
    return band


def dense(band, n, b):
    A = np.zeros((n, n))
    for j in range(n):
        for i in range(j, min(n, j + b + 1)):
            A[i, j] = A[j, i] = band[j, i - j]
    return A


@pytest.mark.parametrize("n,b,tw", [(60, 7, 3), (61, 7, 6), (100, 12, 5), (33, 32, 8), (50, 3, 1), (80, 16, 16),
                                    (40, 50, 4)])
def test_eigenvalues_factors_and_closed_forms(n, b, tw):
    band = sym_band(n, b, seed=n + b)
    bq = min(b, n - 1)
    A = dense(band, n, bq)
    d, e, Q = oracle.sym_reduce(band, n, b, tw, want_q=True)
    T = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
    nA = np.linalg.norm(A, 2)
    assert np.abs(oracle.sym_eigenvalues(d, e) - np.linalg.eigvalsh(A)).max() <= 20 * n * EPS * nA
    assert np.abs(Q.T @ A @ Q - T).max() <= 20 * n * EPS * nA
    assert np.abs(Q.T @ Q - np.eye(n)).max() <= 20 * n * EPS
    assert np.array_equal(Q[:, 0], np.eye(n)[:, 0])
    assert d[0] == A[0, 0]
    assert abs(abs(e[0]) - np.linalg.norm(A[1:bq + 1, 0])) <= 8 * EPS * np.linalg.norm(A)
    assert abs(np.sum(d * d) + 2 * np.sum(e * e) - np.sum(A * A)) <= 20 * n * EPS * np.sum(A * A)


@pytest.mark.parametrize("n,b,tw", [(40, 6, 2), (64, 9, 4), (50, 20, 7)])
def test_unique_up_to_signs_against_lapack_hessenberg(n, b, tw):
    # diagonally dominant bands keep the tridiagonal well away from splitting
    band = sym_band(n, b, seed=3 * n, dominant=True)
    A = dense(band, n, b)
    d, e = oracle.sym_reduce(band, n, b, tw)
    H = scipy.linalg.hessenberg(A)
    assert np.abs(np.abs(d) - np.abs(np.diag(H))).max() <= 1e-12 * np.linalg.norm(A)
    assert np.abs(np.abs(e) - np.abs(np.diag(H, -1))).max() <= 1e-12 * np.linalg.norm(A)


def test_tridiagonal_input_is_returned_bitwise_and_degenerate_shapes():
    n = 30
    band = sym_band(n, 1, seed=5)
    # stored with b = 4: the entries beyond the first sub-diagonal are zero
    wide = np.zeros((n, 5))
    wide[:, :2] = band
    d, e = oracle.sym_reduce(wide, n, 4, 2)
    assert np.array_equal(d, band[:, 0]) and np.array_equal(e, band[:-1, 1])
    d, e = oracle.sym_reduce(band, n, 1, 3)
    assert np.array_equal(d, band[:, 0]) and np.array_equal(e, band[:-1, 1])
    diag = sym_band(7, 0, seed=1)
    d, e = oracle.sym_reduce(diag, 7, 0, 3)
    assert np.array_equal(d, diag[:, 0]) and np.array_equal(e, np.zeros(6))
    for n in (1, 2):
        band = sym_band(n, 3, seed=n)
        d, e = oracle.sym_reduce(band, n, 3, 2)
        A = dense(band, n, min(3, n - 1))
        assert np.array_equal(d, np.diag(A)) and np.array_equal(e, np.diag(A, -1))


def test_tilewidth_only_changes_rounding():
    n, b = 90, 17
    band = sym_band(n, b, seed=11, dominant=True)
    ref = None
    for tw in (1, 3, 8, 16):
        d, e = oracle.sym_reduce(band, n, b, tw)
        cur = np.concatenate([np.abs(d), np.abs(e)])
        if ref is not None:
            assert np.abs(cur - ref).max() <= 1e-12 * np.abs(ref).max()
        ref = cur
