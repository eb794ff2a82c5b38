"""The order in which the back-transformation applies the reflectors.

The oracle accumulates U <- U H (and V <- V H) in the sequential order of the
reduction: stage by stage, sweep by sweep, step by step.  The GPU kernel keeps a
sliding window of one row in registers and, within a stage, takes the steps in
decreasing order and, for each step j, the sweeps in increasing order (the
support p..p+m, p = r + c + j b, then slides by one column per sweep).  Two
reflectors of one side whose supports share a column are taken in the same
relative order by both (same step: by sweep; different steps: the supports can
only meet if the sweep of the larger step comes first), so every entry sees the
same operations in the same order.  Checked here with random reflectors of the
exact geometry, bitwise, including stages with c = 1 and c = 2 and ragged
bottoms; also the order of the two-wave kernel (steps j and j-1 side by side,
the second a few blocks behind, either wave first within a block iteration);
the same function with the steps taken in increasing order must differ (the
check is sharp).
"""
import numpy as np
import pytest


def stages(b, tw):
    out = []
    while b > 1:
        t = min(tw, b - 1)
        out.append((b, t, b - t))
        b -= t
    return out


def steps_of(n, b, tw, c):
    """(r, j, p, m) of every step of a stage, sweep-major."""
    out = []
    for r in range(n - c - 1):
        j = 0
        while True:
            p = r + c + j * b
            m = min(tw, n - 1 - p)
            if m < 1:
                break
            out.append((r, j, p, m))
            j += 1
    return out


def apply(X, p, m, v, tau):
    # plain sequential dot and update, as the oracle does
    for i in range(X.shape[0]):
        w = 0.0
        for t in range(m + 1):
            w = w + X[i, p + t] * v[t]
        tw = tau * w
        for t in range(m + 1):
            X[i, p + t] = X[i, p + t] - tw * v[t]


def two_wave_order(st, n, b, c, tw, trailing_first, blk=8, ahead=16):
    """The order of the two-wave back-transformation: steps j and j-1 (j from the
    last step down, two at a time) on two waves; in block iteration it the first
    wave takes sweeps it*blk .. it*blk + blk - 1 of step j, the second sweeps
    (it - lag)*blk ... of step j-1, lag = max(0, ceil((blk + R - b) / blk)) with
    R = TWM + 1 + ahead (no lag when either step has no sweeps).  The two waves run
    an iteration at the same time, so both orders within an iteration are taken."""
    by = {(r, j): (r, j, p, m) for (r, j, p, m) in st}
    nsteps = 1 + max(j for (_, j, _, _) in st)
    twm = 8 if tw <= 8 else (16 if tw <= 16 else 32)
    R = twm + 1 + ahead
    lag = max(0, -(-(blk + R - b) // blk))
    seq = []
    for j in range(nsteps - 1, -1, -2):
        rca = max(0, n - 1 - c - j * b)
        rcb = max(0, n - 1 - c - (j - 1) * b) if j >= 1 else 0
        la = lag if rca > 0 and rcb > 0 else 0
        its = max(-(-rca // blk), la + -(-rcb // blk))
        for it in range(its):
            blocks = [[by[(r, j)] for r in range(it * blk, (it + 1) * blk) if (r, j) in by],
                      [by[(r, j - 1)] for r in range((it - la) * blk, (it - la + 1) * blk) if r >= 0 and (r, j - 1) in by]]
            if trailing_first:
                blocks.reverse()
            seq += blocks[0] + blocks[1]
    assert sorted(seq) == sorted(st)
    return seq


def run(n, b, tw, order, seed):
    rng = np.random.default_rng(seed)
    X = np.eye(n)
    for (bs, t, c) in stages(b, tw):
        st = steps_of(n, bs, t, c)
        refl = {}
        for (r, j, p, m) in st:
            v = np.concatenate([[1.0], rng.standard_normal(m)])
            refl[(r, j)] = (p, m, v, 2.0 / float(v @ v))
        if order == "sweep-major":
            seq = st
        elif order == "step-desc":
            seq = sorted(st, key=lambda s: (-s[1], s[0]))
        elif order in ("two-wave", "two-wave-trailing-first"):
            seq = two_wave_order(st, n, bs, c, t, order == "two-wave-trailing-first")
        else:  # step ascending: not a valid order when supports of different steps meet
            seq = sorted(st, key=lambda s: (s[1], s[0]))
        for (r, j, p, m) in seq:
            pp, mm, v, tau = refl[(r, j)]
            apply(X, pp, mm, v, tau)
    return X


@pytest.mark.parametrize("n,b,tw", [(40, 6, 5), (37, 7, 3), (30, 5, 2), (45, 9, 4), (33, 8, 8), (25, 3, 1)])
def test_step_descending_order_is_bitwise_the_sequential_one(n, b, tw):
    ref = run(n, b, tw, "sweep-major", seed=n + b)
    got = run(n, b, tw, "step-desc", seed=n + b)
    assert np.array_equal(ref, got)


@pytest.mark.parametrize("order", ["two-wave", "two-wave-trailing-first"])
@pytest.mark.parametrize("n,b,tw", [(40, 6, 5), (37, 7, 3), (30, 5, 2), (45, 9, 4), (33, 8, 8), (25, 3, 1),
                                    (90, 20, 16), (160, 70, 32), (120, 33, 32)])
def test_two_wave_order_is_bitwise_the_sequential_one(n, b, tw, order):
    ref = run(n, b, tw, "sweep-major", seed=n + b)
    got = run(n, b, tw, order, seed=n + b)
    assert np.array_equal(ref, got)


def test_step_ascending_order_differs():
    ref = run(40, 6, 5, "sweep-major", seed=1)
    bad = run(40, 6, 5, "step-asc", seed=1)
    assert not np.array_equal(ref, bad)
