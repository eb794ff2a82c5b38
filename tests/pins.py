"""Independent references used to pin the oracle (test helpers only).

None of these share code with the oracle: they are textbook algorithms written
out from their definitions.
"""
import numpy as np


def band_to_dense(band, n, b):
    """Dense n x n matrix from a LAPACK upper band (n, ldband) array."""
    A = np.zeros((n, n))
    for j in range(n):
        for i in range(max(0, j - b), j + 1):
            A[i, j] = band[j, b + i - j]
    return A


def dense_to_band(A, b, ld=None):
    n = A.shape[0]
    ld = ld or b + 1
    band = np.zeros((n, ld))
    for j in range(n):
        for i in range(max(0, j - b), j + 1):
            band[j, b + i - j] = A[i, j]
    return band


def jacobi_singular_values(A, tol=1e-15, max_sweeps=60):
    """One-sided (Hestenes) Jacobi: rotate column pairs until mutually orthogonal;
    the singular values are then the column norms.  Brute force, O(n^3) per sweep."""
    G = np.array(A, dtype=np.float64, copy=True)
    n = G.shape[1]
    for _ in range(max_sweeps):
        off = 0.0
        for i in range(n - 1):
            for j in range(i + 1, n):
                a = G[:, i] @ G[:, i]
                bb = G[:, j] @ G[:, j]
                g = G[:, i] @ G[:, j]
                if a == 0.0 or bb == 0.0:
                    continue
                rel = abs(g) / np.sqrt(a * bb)
                off = max(off, rel)
                if rel <= tol:
                    continue
                zeta = (bb - a) / (2.0 * g)
                t = np.sign(zeta) / (abs(zeta) + np.sqrt(1.0 + zeta * zeta)) if zeta != 0 else 1.0
                c = 1.0 / np.sqrt(1.0 + t * t)
                s = c * t
                gi = G[:, i].copy()
                G[:, i] = c * gi - s * G[:, j]
                G[:, j] = s * gi + c * G[:, j]
        if off <= tol:
            break
    return np.sort(np.linalg.norm(G, axis=0))[::-1]


def _house_vec(x):
    """Reflector H = I - tau v v^T with H x = beta e1 (returns v, tau, beta)."""
    alpha = x[0]
    sigma = np.linalg.norm(x[1:])
    v = np.zeros_like(x)
    v[0] = 1.0
    if sigma == 0.0:
        return v, 0.0, alpha
    beta = -np.copysign(np.hypot(alpha, sigma), alpha if alpha != 0 else 1.0)
    v[1:] = x[1:] / (alpha - beta)
    return v, (beta - alpha) / beta, beta


def golub_kahan_dense(A):
    """Textbook dense Householder bidiagonalisation (Golub & Van Loan, Alg. 5.4.2):
    alternately annihilate column j below the diagonal and row j right of the
    super-diagonal.  Returns (d, e)."""
    B = np.array(A, dtype=np.float64, copy=True)
    n = B.shape[0]
    for j in range(n):
        v, tau, _ = _house_vec(B[j:, j].copy())
        B[j:, j:] -= tau * np.outer(v, v @ B[j:, j:])
        if j < n - 2:
            v, tau, _ = _house_vec(B[j, j + 1:].copy())
            B[j:, j + 1:] -= tau * np.outer(B[j:, j + 1:] @ v, v)
    return np.diag(B).copy(), np.diag(B, 1).copy()
