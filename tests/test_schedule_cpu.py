"""Exhaustive happens-before check of the sweep schedule the stage kernels run.

Half-step h of sweep r (h = 2j: right task of step j, h = 2j+1: left task) starts
after half-step h-1 of its own sweep and after sweep r-1 has completed h + H
half-steps (or, when sweep r-1 has fewer, after sweep r-1 and every earlier sweep
finished).  Sweep r-i is then only known to have completed h + i (H - 1) + 1
half-steps.  With H = bb_min_lag(c), every pair of half-steps this leaves unordered
must touch disjoint band entries, so the concurrent order gives the sequential
result of Algorithm 1 bit for bit.  The kernels also move the row-k rewrite of a
right task into the next half-step when c == 2 or c >= 4; that variant is checked
the same way, and the check shows why c = 1 and c = 3 must not use it.
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


def unordered_conflicts(n, b, tw, H, defer):
    c = b - tw
    ns = n - c - 1
    lens, sets = [], {}
    for r in range(ns):
        j = 0
        while True:
            k, p, m = geom(n, b, tw, c, r, j)
            if m < 1:
                break
            last = min(p + m + b, n - 1)
            right = {(i, q) for i in range(k, p + m + 1) for q in range(p, p + m + 1)}
            left = {(i, q) for i in range(p, p + m + 1) for q in range(p, last + 1)}
            if defer:
                left |= {(k, q) for q in range(p, p + m + 1)}
            sets[(r, 2 * j)], sets[(r, 2 * j + 1)] = right, left
            j += 1
        lens.append(2 * j)
    full = np.array(lens)
    done = {}  # done[(r, h)][r2]: half-steps of sweep r2 complete before (r, h) starts
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
    bad = set()
    for nodes in touching.values():
        for a in range(len(nodes)):
            for z in range(a + 1, len(nodes)):
                x, y = nodes[a], nodes[z]
                if x[0] == y[0]:
                    continue
                if done[y][x[0]] <= x[1] and done[x][y[0]] <= y[1]:
                    bad.add((x, y))
    return len(bad)


def stages(b, tw):
    out = []
    while b > 1:
        t = min(tw, b - 1)
        out.append((b, t, b - t))
        b -= t
    return out


@pytest.mark.parametrize("n,b,tw", [(120, 24, 1), (100, 12, 3), (90, 16, 5), (80, 10, 2), (70, 9, 4),
                                    (60, 33, 32), (140, 40, 16)])
def test_lag_rule_leaves_only_disjoint_half_steps_concurrent(n, b, tw):
    for bs, t, c in stages(b, tw):
        H = bb.min_lag(c)
        assert unordered_conflicts(n, bs, t, H, defer=False) == 0, (bs, t, c, H)


@pytest.mark.parametrize("c", [1, 2, 3, 4, 5, 8])
@pytest.mark.parametrize("tw", [1, 3, 8])
def test_row_k_deferral_is_safe_exactly_where_the_kernels_use_it(c, tw):
    n, b = 60 + 3 * (c + tw), c + tw
    H = bb.min_lag(c)
    conflicts = unordered_conflicts(n, b, tw, H, defer=True)
    kernel_defers = c == 2 or c >= 4
    if kernel_defers:
        assert conflicts == 0
    else:
        assert conflicts > 0  # the kernels write row k in the same phase here


def test_a_smaller_lag_than_the_minimum_is_unsafe():
    """The check is sharp: one half-step less than bb_min_lag(c) leaves conflicts."""
    for b, tw in [(12, 3), (10, 8), (9, 7)]:
        c = b - tw
        H = bb.min_lag(c)
        assert unordered_conflicts(80, b, tw, H - 1, defer=False) > 0, (b, tw, c, H)


def early_rule_violations(n, b, tw, H, defer):
    """Half-steps whose early loads (right task: rows <= p-2 and row k; left task:
    columns <= p+b-2) could see a value that a sequentially earlier half-step has
    not yet written, when sweep r-1 has completed only h + H - 1 half-steps."""
    c = b - tw
    ns = n - c - 1
    lens, sets, geo = [], {}, {}
    for r in range(ns):
        j = 0
        while True:
            k, p, m = geom(n, b, tw, c, r, j)
            if m < 1:
                break
            last = min(p + m + b, n - 1)
            right = {(i, q) for i in range(k, p + m + 1) for q in range(p, p + m + 1)}
            left = {(i, q) for i in range(p, p + m + 1) for q in range(p, last + 1)}
            if defer:
                left |= {(k, q) for q in range(p, p + m + 1)}
            sets[(r, 2 * j)], sets[(r, 2 * j + 1)] = right, left
            geo[(r, j)] = (k, p, m)
            j += 1
        lens.append(2 * j)
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
    for (r, h), s in sets.items():
        if r == 0:
            continue
        weak = np.zeros(ns, dtype=np.int64)  # guaranteed under the weaker wait
        if h > 0:
            weak = np.maximum(weak, done[(r, h - 1)])
            weak[r] = max(weak[r], h)
        if h + H - 1 > lens[r - 1]:
            weak[:r] = np.maximum(weak[:r], full[:r])
        else:
            weak = np.maximum(weak, done[(r - 1, h + H - 2)])
            weak[r - 1] = max(weak[r - 1], h + H - 1)
        k, p, m = geo[(r, h // 2)]
        if h % 2 == 0:
            early = [(i, q) for (i, q) in s if i <= p - 2 or i == k]
        else:
            early = [(i, q) for (i, q) in s if q <= p + b - 2 and i != k]
        for e in early:
            for (r2, h2) in touching[e]:
                if (r2 < r or (r2 == r and h2 < h)) and weak[r2] <= h2:
                    bad += 1
    return bad


@pytest.mark.parametrize("n,b,tw", [(90, 16, 4), (80, 12, 3), (70, 11, 9), (100, 32, 8), (60, 7, 5), (50, 6, 5)])
def test_early_loads_read_only_final_values(n, b, tw):
    """With one sweep per workgroup the kernels wait first for one half-step less
    than the rule and load part of the window then; every value loaded early must
    already be final in the sequential order."""
    for bs, t, c in stages(b, tw):
        H = bb.min_lag(c)
        assert early_rule_violations(n, bs, t, H, defer=(c == 2 or c >= 4)) == 0, (bs, t, c, H)
