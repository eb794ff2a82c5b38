"""Exhaustive happens-before check of the symmetric chase's sweep schedule.

One task per step (the reflector is applied from both sides inside it).  Step
j of sweep r starts after step j-1 of its sweep and after sweep r-1 completed
j + H steps (or finished, with every earlier sweep).  With H = bb_sym_min_lag(c)
(2 for c >= 2, 3 for c = 1) every pair of steps that this leaves unordered
touches disjoint entries of the stored lower triangle, so the pipelined order
gives the sequential result bit for bit; one step less leaves conflicts.
"""
import numpy as np
import pytest

from paper_2510_12705_amd import bb


def geom(n, b, tw, c, r, j):
    if j == 0:
        k, p = r, r + c
        m = min(r + b, n - 1) - p
    else:
        k = r + c + (j - 1) * b
        p = k + b
        m = min(tw, n - 1 - p)
    return k, p, m


def window(n, b, tw, c, r, j):
    k, p, m = geom(n, b, tw, c, r, j)
    if m < 1:
        return None
    last = min(p + m + b, n - 1)
    s = {(i, q) for q in range(k, p + m + 1) for i in range(max(p, q), p + m + 1)}
    s |= {(i, q) for i in range(p, last + 1) for q in range(p, p + m + 1) if i >= q}
    return s


def unordered_conflicts(n, b, tw, H):
    c = b - tw
    ns = n - c - 1
    lens, sets = [], {}
    for r in range(ns):
        j = 0
        while True:
            w = window(n, b, tw, c, r, j)
            if w is None:
                break
            sets[(r, j)] = w
            j += 1
        lens.append(j)
    full = np.array(lens)
    done = {}
    for r in range(ns):
        for h in range(lens[r]):
            g = np.zeros(ns, dtype=np.int64)
            if h > 0:
                g = np.maximum(g, done[(r, h - 1)])
                g[r] = max(g[r], h)
            if r > 0:
                if h + H > lens[r - 1]:
                    g[:r] = np.maximum(g[:r], full[:r])
                else:
                    g = np.maximum(g, done[(r - 1, h + H - 1)])
                    g[r - 1] = max(g[r - 1], h + H)
            done[(r, h)] = g
    touching = {}
    for node, s in sets.items():
        for e in s:
            touching.setdefault(e, []).append(node)
    bad = 0
    for nodes in touching.values():
        for a in range(len(nodes)):
            for z in range(a + 1, len(nodes)):
                x, y = nodes[a], nodes[z]
                if x[0] != y[0] and done[y][x[0]] <= x[1] and done[x][y[0]] <= y[1]:
                    bad += 1
    return bad


@pytest.mark.parametrize("n,b,tw", [(60, 5, 4), (50, 3, 2), (80, 6, 3), (64, 4, 2), (70, 8, 1), (90, 16, 8)])
def test_sym_lag_is_safe_and_tight(n, b, tw):
    c = b - tw
    H = bb.sym_min_lag(c)
    assert H == (3 if c == 1 else 2)
    assert unordered_conflicts(n, b, tw, H) == 0
    assert unordered_conflicts(n, b, tw, H - 1) > 0


def _py_sym_model_bytes(n, b, elem, tw):
    tot = 0
    bq = min(b, n - 1)
    while bq > 1:
        t = min(tw, bq - 1)
        c = bq - t
        for r in range(n - c - 1):
            j = 0
            while True:
                w = window(n, bq, t, c, r, j)
                if w is None:
                    break
                tot += len(w)
                j += 1
        bq = c
    return 2.0 * tot * elem


@pytest.mark.parametrize("n,b,tw,elem", [(60, 7, 3, 8), (45, 12, 12, 4), (30, 3, 1, 8), (25, 30, 8, 8)])
def test_sym_model_bytes_counts_every_window_entry(n, b, tw, elem):
    assert bb.sym_model_bytes(n, b, elem, tw) == pytest.approx(_py_sym_model_bytes(n, b, elem, tw), rel=1e-12)
