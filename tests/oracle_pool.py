"""Run the CPU oracle on several host cores for the GPU tests' full-size checks.

Test infrastructure only (imports the oracle).  Workers are started with the
"spawn" method and never touch the GPU: they get numpy arrays and return numpy
arrays.
"""
from __future__ import annotations

import hashlib
import json
import multiprocessing as mp
import os
from concurrent.futures import ProcessPoolExecutor

import numpy as np

GOLDEN_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def de_hash(d, e) -> str:
    """SHA-256 of d then e as little-endian float64 (the format of full_size.json)."""
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(d, dtype="<f8").tobytes())
    h.update(np.ascontiguousarray(e, dtype="<f8").tobytes())
    return h.hexdigest()


def golden(name: str):
    """The entry `name` of golden/full_size.json, with its sigma array (or None)."""
    with open(os.path.join(GOLDEN_DIR, "full_size.json")) as f:
        ents = {r["name"]: r for r in json.load(f)["entries"]}
    if name not in ents:
        return None, None
    rec = ents[name]
    sig = None
    if rec.get("sigma_file"):
        sig = np.load(os.path.join(GOLDEN_DIR, rec["sigma_file"]), allow_pickle=False)
    return rec, sig


def _sigma(de):
    import oracle
    d, e = de
    return oracle.singular_values(d, e)


def _reduce_sigma(job):
    import oracle
    band, n, b, tw = job
    d, e = oracle.reduce(band, n, b, tw)
    return oracle.singular_values(d, e)


def _map(fn, items, workers=None):
    items = list(items)
    if not items:
        return []
    workers = workers or max(1, min(16, os.cpu_count() or 1, len(items)))
    if workers == 1:
        return [fn(x) for x in items]
    with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        return list(ex.map(fn, items))


def sigma_many(pairs, workers=None):
    """oracle.singular_values(d, e) for each (d, e) pair."""
    return _map(_sigma, pairs, workers)


def reduce_sigma_many(jobs, workers=None):
    """For each (band, n, b, tw): sigma of the oracle's reduction of that band."""
    return _map(_reduce_sigma, jobs, workers)
