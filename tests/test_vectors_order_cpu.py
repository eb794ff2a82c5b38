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
bottoms; the same function with the steps taken in increasing order must
differ (the check is sharp).
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


def test_step_ascending_order_differs():
    ref = run(40, 6, 5, "sweep-major", seed=1)
    bad = run(40, 6, 5, "step-asc", seed=1)
    assert not np.array_equal(ref, bad)
