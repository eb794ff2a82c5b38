"""The paper's accuracy experiment (Sec. V-A) on this library.

Matrices with known singular values: A = U diag(sigma) V^T with Haar-random
orthogonal U, V and a prescribed spectrum in [0, 1] -- arithmetic (uniform
spacing), logarithmic decay, or drawn from the quarter-circle law -- are
reduced to an upper band of b super-diagonals by the classical block
Householder reduction in FP64 on the host (the first stage of the two-stage
SVD; here part of the input recipe, not of the path under test).  The band then
goes through the GPU band -> bidiagonal reduction stored in FP64, FP32 or FP16,
the singular values of the bidiagonal come from ``bb_bidiag_sigma`` (FP64), and
the error is the paper's ``||sigma_hat - sigma|| / ||sigma||`` against the
prescribed sigma (the max |dsigma| / sigma_max is reported beside it).

    python -m paper_2510_12705_amd.accuracy [--n 1024,2048] [--b 32,128] [--trials 10]

Only the first stage uses the host; nothing here calls a CPU version of the
reduction.
"""
from __future__ import annotations

import argparse
import math
import sys
import time

import numpy as np

SPECTRA = ("arithmetic", "logarithmic", "quarter-circle")
LOG_DECADES = 6.0  # logarithmic decay from 1 to 1e-6


def spectrum(kind: str, n: int, rng: np.random.Generator) -> np.ndarray:
    """Prescribed singular values in [0, 1], descending."""
    if kind == "arithmetic":
        s = np.arange(n, 0, -1, dtype=np.float64) / n
    elif kind == "logarithmic":
        s = 10.0 ** (-LOG_DECADES * np.arange(n, dtype=np.float64) / max(n - 1, 1))
    elif kind == "quarter-circle":
        # density (4/pi) sqrt(1 - x^2) on [0, 1]; CDF F(x) = (2/pi)(x sqrt(1 - x^2) + asin x),
        # inverted by bisection at sorted uniform draws
        u = np.sort(rng.uniform(0.0, 1.0, n))[::-1]
        lo, hi = np.zeros(n), np.ones(n)
        for _ in range(60):
            mid = 0.5 * (lo + hi)
            F = (2.0 / math.pi) * (mid * np.sqrt(1.0 - mid * mid) + np.arcsin(mid))
            lo = np.where(F < u, mid, lo)
            hi = np.where(F < u, hi, mid)
        s = 0.5 * (lo + hi)
    else:
        raise ValueError(kind)
    return s


def haar_orthogonal(n: int, rng: np.random.Generator) -> np.ndarray:
    q, r = np.linalg.qr(rng.standard_normal((n, n)))
    return q * np.sign(np.diag(r))


def dense_to_band(A: np.ndarray, b: int) -> np.ndarray:
    """Block Householder reduction of a dense n x n matrix to upper band form with b
    super-diagonals, in FP64: for each block column k, a QR of the panel A[k:, k:k+b]
    annihilates it below its diagonal block (its Q^T is applied to the columns to the
    right), then an LQ of the row panel A[k:k+b, k+b:] (a QR of its transpose)
    annihilates it right of a lower-triangular block (its Q applied to the rows
    below).  Returns the (n, b+1) LAPACK upper band of the result."""
    from scipy.linalg import lapack
    A = np.array(A, dtype=np.float64, order="F", copy=True)
    n = A.shape[0]
    for k in range(0, n, b):
        kb = min(k + b, n)
        w = kb - k
        qr, tau, _, info = lapack.dgeqrf(A[k:, k:kb], lwork=max(1, 64 * w))
        assert info == 0
        if kb < n:
            C = np.asfortranarray(A[k:, kb:])
            A[k:, kb:] = lapack.dormqr(b"L", b"T", qr[:, :len(tau)], tau, C, max(1, 64 * C.shape[1]))[0]
        A[k:, k:kb] = 0.0
        rr = min(n - k, w)
        A[k:k + rr, k:kb] = np.triu(qr[:rr, :])
        if kb < n:
            X = np.asfortranarray(A[k:kb, kb:].T)
            qr2, tau2, _, info = lapack.dgeqrf(X, lwork=max(1, 64 * w))
            assert info == 0
            C = np.asfortranarray(A[kb:, kb:])
            A[kb:, kb:] = lapack.dormqr(b"R", b"N", qr2[:, :len(tau2)], tau2, C, max(1, 64 * C.shape[0]))[0]
            A[k:kb, kb:] = 0.0
            rr = min(n - kb, w)
            A[k:kb, kb:kb + rr] = np.triu(qr2[:rr, :]).T
    band = np.zeros((n, b + 1))
    for j in range(n):
        i0 = max(0, j - b)
        band[j, b - (j - i0):] = A[i0:j + 1, j]
    return band


def test_matrix(kind: str, n: int, b: int, seed: int):
    """(band, sigma) of one instance: the FP64 band of U diag(sigma) V^T."""
    rng = np.random.default_rng(seed)
    s = spectrum(kind, n, rng)
    U = haar_orthogonal(n, rng)
    V = haar_orthogonal(n, rng)
    A = (U * s) @ V.T
    return dense_to_band(A, b), s


def gpu_sigma(band: np.ndarray, n: int, b: int, dtype_name: str):
    import torch

    from . import bb
    dt = {"fp64": torch.float64, "fp32": torch.float32, "fp16": torch.float16}[dtype_name]
    t = torch.from_numpy(np.ascontiguousarray(band)).cuda().to(dt)
    d, e = bb.bb_reduce(t, n, b)
    s = bb.bidiag_sigma(d, e)
    st = bb.stream_status()
    if st != 0:
        raise RuntimeError(bb.bb_error_string(st))
    return s.cpu().numpy()


def errors(s_hat: np.ndarray, s: np.ndarray):
    return (float(np.linalg.norm(s_hat - s) / np.linalg.norm(s)), float(np.max(np.abs(s_hat - s)) / s[0]))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", default="1024,2048")
    ap.add_argument("--b", default="32,128")
    ap.add_argument("--trials", type=int, default=10)
    args = ap.parse_args()
    ns = [int(x) for x in args.n.split(",")]
    bs = [int(x) for x in args.b.split(",")]
    print("| n | b | spectrum | FP64 median / max rel. error | FP32 median / max | FP16 median / max |")
    print("|---:|---:|---|---|---|---|")
    for n in ns:
        for b in bs:
            for kind in SPECTRA:
                res = {p: [] for p in ("fp64", "fp32", "fp16")}
                t0 = time.perf_counter()
                for trial in range(args.trials):
                    band, s = test_matrix(kind, n, b, seed=1000 * n + 10 * b + trial)
                    for p in res:
                        res[p].append(errors(gpu_sigma(band, n, b, p), s)[0])
                cells = ["%.2e / %.2e" % (float(np.median(res[p])), float(np.max(res[p]))) for p in res]
                print("| %d | %d | %s | %s |  <!-- %.1f s -->" % (n, b, kind, " | ".join(cells),
                                                                 time.perf_counter() - t0), flush=True)


if __name__ == "__main__":
    main()
    sys.exit(0)
