"""CPU oracle for band -> bidiagonal reduction (bulge chasing).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the GPU library and never imports it.

Contents
  * ``reduce``            -- the plain FP64 sequential bulge chase (C, ``bb_oracle.c``),
                             following Algorithm 1 of the paper stage by stage,
                             sweep by sweep, step by step.
  * ``reduce_pipelined``  -- the same arithmetic run in a random order allowed by a
                             half-step dependency rule (host race detector).
  * ``reduce_dense_full`` -- an independent pure-Python coding on a dense matrix that
                             applies every reflector to all rows and columns (no index
                             ranges at all), for pinning the band code's ranges.
  * ``nrm2``              -- the C oracle's norm on its own, for its pins.
  * ``sym_reduce``        -- the symmetric variant: a symmetric band reduced to
                             tridiagonal by the same chase with one reflector per
                             step applied from both sides (C, ``bb_oracle.c``).
  * ``sym_eigenvalues``   -- eigenvalues of a symmetric tridiagonal, LAPACK dsterf.
  * ``singular_values``   -- sigma of a bidiagonal (d, e) as the non-negative
                             eigenvalues of its Golub-Kahan (TGK) tridiagonal, via
                             LAPACK dsterf; the paper uses LAPACK BDSDC for this step
                             (Sec. V-A), which SciPy does not wrap.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bb_oracle.c")
_LIB = os.path.join(_HERE, "_build", "libbb_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (no FMA contraction).  Returns the .so path."""
    os.makedirs(os.path.dirname(_LIB), exist_ok=True)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-fopenmp",
                               "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        i64 = ctypes.c_int64
        lib.bbo_reduce.argtypes = [i64, i64, i64, dp, i64, dp, dp, dp, dp, ctypes.c_int]
        lib.bbo_reduce.restype = ctypes.c_int
        lib.bbo_reduce_pipelined.argtypes = [i64, i64, i64, dp, i64, dp, dp,
                                             ctypes.POINTER(ctypes.c_int), ctypes.c_uint64]
        lib.bbo_reduce_pipelined.restype = ctypes.c_int
        lib.bbo_reduce_wavefront.argtypes = [i64, i64, i64, dp, i64, dp, dp, ctypes.POINTER(ctypes.c_int),
                                             ctypes.c_int, i64, i64, ctypes.POINTER(ctypes.c_int)]
        lib.bbo_reduce_wavefront.restype = ctypes.c_int
        lib.bbo_nrm2.argtypes = [dp, i64]
        lib.bbo_nrm2.restype = ctypes.c_double
        lib.bbo_sym_reduce.argtypes = [i64, i64, i64, dp, i64, dp, dp, dp]
        lib.bbo_sym_reduce.restype = ctypes.c_int
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if a is not None else None


def reduce(band: np.ndarray, n: int, b: int, tw: int, want_uv: bool = False, rev: bool = False):
    """Sequential FP64 reduction of a LAPACK upper band to bidiagonal (d, e).

    ``band`` is an (n, ldband) C-ordered float64 array, i.e. the column-major
    LAPACK band with A(i, j) = band[j, b + i - j] for max(0, j-b) <= i <= j.
    ``tw`` is the inner tilewidth TW.  With ``want_uv`` also returns U, V with
    U^T A V = bidiag(d, e) (dense, n x n).  ``rev`` reverses every dot product.
    """
    lib = _load()
    band = np.ascontiguousarray(band, dtype=np.float64)
    ldband = band.shape[1] if band.ndim == 2 else b + 1
    d = np.zeros(max(n, 1))
    e = np.zeros(max(n - 1, 1))
    U = V = None
    if want_uv:
        U = np.zeros((n, n), order="F")
        V = np.zeros((n, n), order="F")
    rc = lib.bbo_reduce(n, b, tw, _dp(band), ldband, _dp(d), _dp(e), _dp(U), _dp(V), int(rev))
    if rc != 0:
        raise ValueError("bbo_reduce failed with code %d" % rc)
    d, e = d[:n], e[:max(n - 1, 0)]
    if want_uv:
        return d, e, U, V
    return d, e


def sym_reduce(band: np.ndarray, n: int, b: int, tw: int, want_q: bool = False):
    """Sequential FP64 reduction of a symmetric band (lower layout: an (n, ldband)
    C-ordered array with A(i, j) = band[j, i - j] for 0 <= i - j <= b) to
    tridiagonal (d, e); with ``want_q`` also Q with Q^T A Q = tridiag(d, e)."""
    lib = _load()
    band = np.ascontiguousarray(band, dtype=np.float64)
    ldband = band.shape[1] if band.ndim == 2 else b + 1
    d = np.zeros(max(n, 1))
    e = np.zeros(max(n - 1, 1))
    Q = np.zeros((n, n), order="F") if want_q else None
    rc = lib.bbo_sym_reduce(n, b, tw, _dp(band), ldband, _dp(d), _dp(e), _dp(Q))
    if rc != 0:
        raise ValueError("bbo_sym_reduce failed with code %d" % rc)
    d, e = d[:n], e[:max(n - 1, 0)]
    return (d, e, Q) if want_q else (d, e)


def sym_eigenvalues(d, e):
    """Eigenvalues (ascending) of the symmetric tridiagonal with diagonal d and
    off-diagonal e, by LAPACK dsterf."""
    from scipy.linalg import lapack
    d = np.array(d, dtype=np.float64)
    if len(d) == 0:
        return d
    w, info = lapack.dsterf(d.copy(), np.array(e, dtype=np.float64).copy())
    if info != 0:
        raise RuntimeError("dsterf failed: %d" % info)
    return np.sort(w)


def nrm2(x) -> float:
    """The C oracle's Euclidean norm (LAPACK >= 3.10 xNRM2) of a float64 vector."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    return float(_load().bbo_nrm2(_dp(x), x.shape[0]))


def reduce_pipelined(band: np.ndarray, n: int, b: int, tw: int, lag, seed: int):
    """Run the reduction in a random order allowed by the half-step lag rule ``lag``
    (a triple: H for c == 1, c == 2, c >= 3).  Raises on deadlock."""
    lib = _load()
    band = np.ascontiguousarray(band, dtype=np.float64)
    d = np.zeros(max(n, 1))
    e = np.zeros(max(n - 1, 1))
    lg = (ctypes.c_int * 3)(*[int(x) for x in lag])
    rc = lib.bbo_reduce_pipelined(n, b, tw, _dp(band), band.shape[1], _dp(d), _dp(e), lg, seed)
    if rc != 0:
        raise RuntimeError("bbo_reduce_pipelined failed with code %d" % rc)
    return d[:n], e[:max(n - 1, 0)]


# Half-step lags of the dependency rule (Sec. III-A): H for c == 1, c == 2, c >= 3.
DEFAULT_LAG = (4, 3, 2)


def reduce_wavefront(band: np.ndarray, n: int, b: int, tw: int, threads: int = 0, group: int = 1,
                     lag=DEFAULT_LAG, max_stages: int = 0):
    """The reduction as a wavefront over host threads (the multi-core CPU
    baseline), ``group`` consecutive sweeps per thread at a time; bitwise equal
    to ``reduce``.  ``max_stages`` > 0 stops after that many stages (a timing
    sample).  Returns (d, e, threads used)."""
    lib = _load()
    band = np.ascontiguousarray(band, dtype=np.float64)
    d = np.zeros(max(n, 1))
    e = np.zeros(max(n - 1, 1))
    lg = (ctypes.c_int * 3)(*[int(x) for x in lag])
    used = ctypes.c_int(0)
    rc = lib.bbo_reduce_wavefront(n, b, tw, _dp(band), band.shape[1], _dp(d), _dp(e), lg, int(threads),
                                  int(group), int(max_stages), ctypes.byref(used))
    if rc != 0:
        raise ValueError("bbo_reduce_wavefront failed with code %d" % rc)
    return d[:n], e[:max(n - 1, 0)], used.value


# ----------------------------------------------------------------------------
# Independent dense coding (pure Python floats; IEEE double, left-to-right sums,
# no fused multiply-add), same Householder convention and the same step order.
# ----------------------------------------------------------------------------

_TSML, _TBIG, _SSML, _SBIG = 2.0 ** -511, 2.0 ** 486, 2.0 ** 537, 2.0 ** -538


def _nrm2(xs):
    """Reference LAPACK (>= 3.10) xNRM2: Blue's algorithm, Anderson's constants."""
    notbig = True
    asml = amed = abig = 0.0
    for x in xs:
        ax = abs(x)
        if ax > _TBIG:
            y = ax * _SBIG
            abig = abig + y * y
            notbig = False
        elif ax < _TSML:
            if notbig:
                y = ax * _SSML
                asml = asml + y * y
        else:
            amed = amed + ax * ax
    if abig > 0.0:
        if amed > 0.0 or amed != amed:
            abig = abig + (amed * _SBIG) * _SBIG
        scl, sumsq = 1.0 / _SBIG, abig
    elif asml > 0.0:
        if amed > 0.0 or amed != amed:
            amed = math.sqrt(amed)
            asml = math.sqrt(asml) / _SSML
            ymin, ymax = (amed, asml) if asml > amed else (asml, amed)
            q = ymin / ymax
            scl, sumsq = 1.0, ymax * ymax * (1.0 + q * q)
        else:
            scl, sumsq = 1.0 / _SSML, asml
    else:
        scl, sumsq = 1.0, amed
    return scl * math.sqrt(sumsq)


def _hypot2(a, b):
    xa, ya = abs(a), abs(b)
    w, z = max(xa, ya), min(xa, ya)
    if z == 0.0:
        return w
    q = z / w
    return w * math.sqrt(1.0 + q * q)


_SAFMIN = 2.2250738585072014e-308 / 2.220446049250313e-16


def _house(x):
    """LAPACK xLARFG, including its rescaling when |beta| < safmin."""
    x = list(x)
    alpha = x[0]
    xn = _nrm2(x[1:])
    if xn == 0.0:
        return [1.0] + [0.0] * (len(x) - 1), 0.0, alpha
    h = _hypot2(alpha, xn)
    beta = -h if alpha >= 0.0 else h
    knt = 0
    if abs(beta) < _SAFMIN:
        rs = 1.0 / _SAFMIN
        while True:
            knt += 1
            x[1:] = [t * rs for t in x[1:]]
            beta = beta * rs
            alpha = alpha * rs
            if not (abs(beta) < _SAFMIN and knt < 20):
                break
        xn = _nrm2(x[1:])
        h = _hypot2(alpha, xn)
        beta = -h if alpha >= 0.0 else h
    scal = 1.0 / (alpha - beta)
    tau = (beta - alpha) / beta
    v = [1.0] + [t * scal for t in x[1:]]
    for _ in range(knt):
        beta = beta * _SAFMIN
    return v, tau, beta


def stage_plan(b: int, tw_max: int):
    """(b_s, tw_s, c_s) for each bandwidth-reduction stage (Alg. 1 outer loop)."""
    out = []
    while b > 1:
        tw = min(tw_max, b - 1)
        out.append((b, tw, b - tw))
        b -= tw
    return out


def reduce_dense_full(A, b: int, tw_max: int):
    """Dense chase applying every reflector to ALL rows / columns (tiny n only).

    ``A`` is a dense n x n array (upper banded).  Returns the final dense matrix
    as a list of lists; it must be exactly bidiagonal."""
    n = len(A)
    M = [[float(A[i][j]) for j in range(n)] for i in range(n)]
    b = min(b, n - 1) if n > 0 else 0
    for (bs, tw, c) in stage_plan(b, tw_max):
        r = 0
        while r + c + 1 <= n - 1:
            j = 0
            while True:
                if j == 0:
                    k, p = r, r + c
                    m = min(r + bs, n - 1) - p
                else:
                    k = r + c + (j - 1) * bs
                    p = k + bs
                    m = min(tw, n - 1 - p)
                if m < 1:
                    break
                v, tau, beta = _house([M[k][p + t] for t in range(m + 1)])
                M[k][p] = beta
                for t in range(1, m + 1):
                    M[k][p + t] = 0.0
                if tau != 0.0:
                    for i in range(n):
                        if i == k:
                            continue
                        w = 0.0
                        for t in range(m + 1):
                            w = w + M[i][p + t] * v[t]
                        tw_ = tau * w
                        for t in range(m + 1):
                            M[i][p + t] = M[i][p + t] - tw_ * v[t]
                v, tau, beta = _house([M[p + t][p] for t in range(m + 1)])
                M[p][p] = beta
                for t in range(1, m + 1):
                    M[p + t][p] = 0.0
                if tau != 0.0:
                    for q in range(n):
                        if q == p:
                            continue
                        w = 0.0
                        for t in range(m + 1):
                            w = w + v[t] * M[p + t][q]
                        tw_ = tau * w
                        for t in range(m + 1):
                            M[p + t][q] = M[p + t][q] - tw_ * v[t]
                j += 1
            r += 1
    return M


def singular_values(d, e) -> np.ndarray:
    """sigma(B) for upper bidiagonal B = bidiag(d, e), descending.

    The 2n x 2n Golub-Kahan tridiagonal with zero diagonal and off-diagonal
    (d0, e0, d1, e1, ..., d_{n-1}) has eigenvalues +-sigma_i; its eigenvalues are
    computed by LAPACK dsterf and the n largest are returned."""
    from scipy.linalg import lapack
    d = np.asarray(d, dtype=np.float64)
    e = np.asarray(e, dtype=np.float64)
    n = d.shape[0]
    if n == 0:
        return np.zeros(0)
    off = np.zeros(2 * n - 1)
    off[0::2] = d
    off[1::2] = e[: n - 1]
    w, info = lapack.dsterf(np.zeros(2 * n), off)
    if info != 0:
        raise RuntimeError("dsterf info=%d" % info)
    return np.sort(w)[::-1][:n].clip(min=0.0)
