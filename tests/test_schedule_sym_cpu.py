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


def _schedule(n, b, tw, H):
    """Steps, their entry sets and, per step, the completed-step vectors it is
    guaranteed under the full rule (done) and under the rule one step weaker
    (weak: sweep r-1 completed j + H - 1 steps)."""
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
    done, weak = {}, {}
    for r in range(ns):
        for h in range(lens[r]):
            g = np.zeros(ns, dtype=np.int64)
            if h > 0:
                g = np.maximum(g, done[(r, h - 1)])
                g[r] = max(g[r], h)
            gw = g.copy()
            if r > 0:
                if h + H > lens[r - 1]:
                    g[:r] = np.maximum(g[:r], full[:r])
                else:
                    g = np.maximum(g, done[(r - 1, h + H - 1)])
                    g[r - 1] = max(g[r - 1], h + H)
                if h + H - 1 > lens[r - 1]:
                    gw[:r] = np.maximum(gw[:r], full[:r])
                else:
                    gw = np.maximum(gw, done[(r - 1, h + H - 2)])
                    gw[r - 1] = max(gw[r - 1], h + H - 1)
            done[(r, h)] = g
            weak[(r, h)] = gw
    return sets, done, weak


def early_end(b, c):
    """Rows below the block that the kernel loads before the full wait: i < p + early_end."""
    return 2 * b - 1 if c == 1 else b - 1


def early_violations(n, b, tw, H, extra_rows=0):
    """Entries the kernel reads before the full wait (column k, the columns left of the
    block, the block, the rows below it up to p + early_end - 1 + extra_rows) that an
    earlier step of another sweep may still write under the weaker guarantee."""
    c = b - tw
    sets, done, weak = _schedule(n, b, tw, H)
    touching = {}
    for node, s in sets.items():
        for e in s:
            touching.setdefault(e, []).append(node)
    bad = 0
    for (r, j), s in sets.items():
        k, p, m = geom(n, b, tw, c, r, j)
        gw = weak[(r, j)]
        for (i, q) in s:
            if i > p + m and i - p >= early_end(b, c) + extra_rows:
                continue  # loaded after the full wait
            for x in touching[(i, q)]:
                if x < (r, j) and x[0] != r and gw[x[0]] <= x[1]:
                    bad += 1
                    break
    return bad


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


@pytest.mark.parametrize("n,b,tw", [(60, 5, 4), (50, 3, 2), (80, 6, 3), (64, 4, 2), (70, 8, 1), (90, 16, 8),
                                    (120, 24, 8), (100, 12, 4), (60, 9, 8), (75, 10, 9), (40, 2, 1)])
def test_sym_early_loads_are_final_and_the_bound_is_tight(n, b, tw):
    """The two-part wait: what the kernel loads before the full wait is final once
    sweep r-1 has completed one step less than the rule asks; one more row below
    the block is not (for some step), so the bound is the largest safe one."""
    c = b - tw
    H = bb.sym_min_lag(c)
    assert early_violations(n, b, tw, H) == 0
    assert early_violations(n, b, tw, H, extra_rows=1) > 0


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
