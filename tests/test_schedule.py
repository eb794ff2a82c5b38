"""The GPU scheduler's half-step lag rule, checked by brute force on the CPU.

For every pair of tasks (sweep r1, half-step h1) and (r2, h2), r1 < r2, whose
windows share an element, the rule must force (r1, h1) to finish before
(r2, h2) starts.  Element sets are computed here from the step geometry of
Algorithm 1 directly (rows/columns each task reads and writes), independently
of the library; the lag values come from the library's planner.  The paper's
own separation argument (Sec. III-A) is the full-step version of this check.
"""
import pytest

bb = pytest.importorskip("paper_2510_12705_amd.bb")


def _tasks(n, b, tw, c):
    sweeps = []
    r = 0
    while r + c + 1 <= n - 1:
        ts = []
        j = 0
        while True:
            if j == 0:
                k, p = r, r + c
                m = min(r + b, n - 1) - p
            else:
                k = r + c + (j - 1) * b
                p = k + b
                m = min(tw, n - 1 - p)
            if m < 1:
                break
            right = {(k, q) for q in range(p, p + m + 1)}
            right |= {(i, q) for i in range(k + 1, p + m + 1) for q in range(p, p + m + 1)}
            L = min(p + m + b, n - 1)
            left = {(i, q) for i in range(p, p + m + 1) for q in range(p, L + 1)}
            ts += [right, left]
            j += 1
        sweeps.append(ts)
        r += 1
    return sweeps


def _first_violation(sweeps, H):
    """Half-step h of sweep r waits for sweep r-1 to complete h+H half-steps or be DONE
    (DONE: all its half-steps ran and sweep r-2 is DONE)."""
    for r2 in range(1, len(sweeps)):
        for h2 in range(len(sweeps[r2])):
            h = h2
            for r1 in range(r2 - 1, -1, -1):
                need = h + H
                if need > len(sweeps[r1]):
                    break  # waits for DONE of r1: everything up to r1 has finished
                for h1 in range(need, len(sweeps[r1])):
                    if sweeps[r1][h1] & sweeps[r2][h2]:
                        return (r1, h1, r2, h2)
                h = need - 1
    return None


CASES = [(n, b, tw) for n in (23, 37) for b in (3, 4, 6, 9, 12) for tw in range(1, b)]


@pytest.mark.parametrize("n,b,tw", CASES)
def test_library_lag_is_safe(n, b, tw):
    c = b - tw
    H = bb.min_lag(c)
    assert _first_violation(_tasks(n, b, tw, c), H) is None


@pytest.mark.parametrize("n,b,tw", [(37, 9, 6), (37, 9, 7), (37, 9, 8), (37, 12, 2)])
def test_library_lag_is_tight(n, b, tw):
    c = b - tw
    H = bb.min_lag(c)
    assert _first_violation(_tasks(n, b, tw, c), H - 1) is not None


def test_paper_three_cycle_rule_is_safe():
    """Sec. III-A: three full cycles (H = 6 half-steps) always suffice."""
    for (n, b, tw) in [(30, 5, 4), (30, 7, 2), (30, 4, 3)]:
        assert _first_violation(_tasks(n, b, tw, b - tw), 6) is None
