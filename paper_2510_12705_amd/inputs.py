"""Seeded synthetic band matrices shaped like the paper's workloads.

This module holds input generation only -- no arithmetic of the reduction --
so that the GPU path and the CPU oracle can be fed identical inputs.

Layout of every band returned here: an (n, b+1) C-ordered float64 array that
is the column-major LAPACK upper band, A(i, j) = band[j, b + i - j] for
max(0, j-b) <= i <= j.  Entries that would lie above row 0 are zero.

Recipes (entries drawn column by column, b+1 values per column):
  * ``normal``  : i.i.d. N(0, 1)
  * ``uniform`` : i.i.d. U[-1, 1]
  * ``graded``  : ``normal`` with column j scaled by 10^(-6 j / n)
The paper evaluates on synthetic matrices only (Sec. V); n ranges over
1024 .. 32768 and bandwidths 32 .. 512 there.
"""
from __future__ import annotations

import math

import numpy as np


def _mask_top(band: np.ndarray, b: int) -> np.ndarray:
    # band[j, off] holds row i = j - b + off; rows < 0 do not exist
    n = band.shape[0]
    for j in range(min(b, n)):
        band[j, : b - j] = 0.0
    return band


def band_normal(n: int, b: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return _mask_top(rng.standard_normal((n, b + 1)), b)


def band_uniform(n: int, b: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return _mask_top(rng.uniform(-1.0, 1.0, (n, b + 1)), b)


def band_graded(n: int, b: int, seed: int) -> np.ndarray:
    band = band_normal(n, b, seed)
    scale = 10.0 ** (-6.0 * np.arange(n) / max(n, 1))
    return band * scale[:, None]


def seed_for_bandwidth_sweep(b: int) -> int:
    return 40 + int(round(math.log2(b)))


# Named workloads: (description, n, b, generator, seed)
WORKLOADS = {
    "n512_b32": ("n=512, b=32, N(0,1) band", 512, 32, band_normal, 1),
    "n8192_b64": ("n=8192, b=64, N(0,1) band", 8192, 64, band_normal, 2),
    "n8192_b64_graded": ("n=8192, b=64, N(0,1) band, column j scaled by 10^(-6j/n)", 8192, 64, band_graded, 2),
    "n32768_b128": ("n=32768, b=128, N(0,1) band", 32768, 128, band_normal, 3),
}
for _b in (16, 32, 64, 128, 256):
    WORKLOADS["n16384_b%d_uniform" % _b] = ("n=16384, b=%d, U[-1,1] band" % _b, 16384, _b, band_uniform,
                                            seed_for_bandwidth_sweep(_b))


def workload(name: str) -> np.ndarray:
    _, n, b, gen, seed = WORKLOADS[name]
    return gen(n, b, seed)


def ragged_batch(count: int = 512, seed: int = 5, n_lo: int = 256, n_hi: int = 4096,
                 bands=(16, 32, 64)):
    """Ragged batch: n_i = floor(exp(U(ln n_lo, ln n_hi))), b_i uniform from
    ``bands``, then the N(0,1) entries of each matrix in order.  Returns a list
    of (n_i, b_i, band_i float64)."""
    rng = np.random.default_rng(seed)
    ns = np.floor(np.exp(rng.uniform(math.log(n_lo), math.log(n_hi), count))).astype(np.int64)
    bs = rng.choice(np.asarray(bands, dtype=np.int64), count)
    out = []
    for n, b in zip(ns.tolist(), bs.tolist()):
        out.append((n, b, _mask_top(rng.standard_normal((n, b + 1)), b)))
    return out
