"""Binomial checkpointing schedule (host logic, no GPU)."""
import itertools
from functools import lru_cache

import pytest

from paper_2505_20911_amd import revolve


def brute_force_min_advances(l, s):
    """Exhaustive minimum over every recursive split sequence (tiny l, s)."""
    @lru_cache(maxsize=None)
    def T(l, s):
        if l == 1:
            return 0
        if s == 0:
            return l * (l - 1) // 2
        return min(m + T(l - m, s - 1) + T(m, s) for m in range(1, l))
    return T(l, s)


@pytest.mark.parametrize("l,s", [(1, 0), (2, 1), (5, 0), (7, 2), (10, 3), (20, 4), (33, 5), (60, 3)])
def test_schedule_is_optimal_and_valid(l, s):
    acts = revolve.schedule(l, s)
    assert revolve.count_advances(acts) == revolve.optimal_advances(l, s) == brute_force_min_advances(l, s)
    # simulate: every step reversed once, in order l..1, from the right state,
    # never more than s snapshots held
    cur, held, reversed_steps = 0, {}, []
    for a in acts:
        if a[0] == "advance":
            assert a[1] == cur
            cur += 1
        elif a[0] == "store":
            assert a[2] == cur and a[1] not in held
            held[a[1]] = cur
            assert len(held) <= s
        elif a[0] == "restore":
            cur = 0 if a[1] == -1 else held[a[1]]
            assert cur == a[2]
        elif a[0] == "free":
            del held[a[1]]
        elif a[0] == "reverse":
            assert cur == a[1] - 1
            reversed_steps.append(a[1])
            cur = None  # the reversal consumes the current state
    assert reversed_steps == list(range(l, 0, -1))


def test_closed_form_matches_recursion():
    for s in range(0, 8):
        for l in range(1, 150):
            assert revolve.optimal_advances(l, s) == revolve.binomial_closed_form(l, s)
    # 400 steps, 20 snapshot buffers beside x_0 (21 counting it)
    assert revolve.optimal_advances(400, 20) == 924
    assert revolve.binomial_closed_form(400, 19) == 947


def test_every_reversal_is_followed_by_a_restore():
    """The reverse sweep leaves the current state at the step's input (it
    recomputes only the stage inputs it needs), which is sound only because a
    reversal is never followed by an advance or a store before a restore."""
    for l in range(1, 60):
        for s in range(1, 12):
            acts = revolve.schedule(l, s)
            for a, b in zip(acts, acts[1:]):
                if a[0] == "reverse":
                    assert b[0] in ("restore", "free"), (l, s, a, b)
            k = 0
            while k < len(acts):
                if acts[k][0] == "free":
                    assert k + 1 < len(acts) and acts[k + 1][0] == "restore", (l, s, acts[k:k + 2])
                k += 1
