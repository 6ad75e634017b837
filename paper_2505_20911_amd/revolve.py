"""Binomial (revolve-style) checkpointing schedule for reversing a chain of
time steps with a bounded number of state snapshots.

Model.  The state x_0 is held by the caller and is always restorable.  There
are ``slots`` further snapshot buffers.  Reversing step n (x_{n-1} -> x_n)
needs x_{n-1} as the *current* state; it re-runs that one step internally to
tape the stage inputs (that re-run is part of the reversal and is not counted
as an advance).  ``advance`` moves the current state forward one step at a
time and is what the schedule minimises.

Recursion (Griewank & Walther, "Algorithm 799: revolve", ACM TOMS 2000): to
reverse l steps starting from a restorable state with s free slots, advance m
steps, store, reverse the last l - m steps with s - 1 slots, free the slot,
then reverse the first m steps with s slots:
    T(1, s) = 0,  T(l, 0) = l (l - 1) / 2,
    T(l, s) = min_{1 <= m < l} m + T(l - m, s - 1) + T(m, s).
The split is taken from this table directly (exact optimum of the model);
the binomial closed form is checked against it in the tests.
"""
from __future__ import annotations

from functools import lru_cache


@lru_cache(maxsize=None)
def _table(l: int, s: int):
    """(T(l, s), best first split m) for l >= 1."""
    if l == 1:
        return 0, 0
    if s == 0:
        return l * (l - 1) // 2, 0
    best, arg = None, 0
    for m in range(1, l):
        c = m + _table(l - m, s - 1)[0] + _table(m, s)[0]
        if best is None or c < best:
            best, arg = c, m
    return best, arg


def optimal_advances(l: int, s: int) -> int:
    """Minimal number of single-step advances to reverse l steps with s slots."""
    import sys
    sys.setrecursionlimit(max(10000, sys.getrecursionlimit()))
    for ll in range(1, l + 1):  # fill bottom-up to keep the recursion shallow
        for ss in range(0, s + 1):
            _table(ll, ss)
    return _table(l, s)[0]


def schedule(l: int, s: int):
    """Action list for reversing steps l..1 with s snapshot slots.

    Actions: ("advance", n) -- current state x_n -> x_{n+1};
             ("store", slot, n) -- copy current x_n into slot;
             ("restore", slot, n) -- current <- slot (holding x_n); slot -1 is x_0;
             ("reverse", n) -- reverse step n (current state is x_{n-1});
             ("free", slot).
    """
    optimal_advances(l, s)
    actions = []
    free = list(range(s))[::-1]

    def rev(start: int, length: int, slot: int, nfree: int):
        # current state is x_start (held in `slot`, -1 = caller's x_0)
        if length == 1:
            actions.append(("reverse", start + 1))
            return
        if nfree == 0:
            for j in range(length, 0, -1):
                if j != length:
                    actions.append(("restore", slot, start))
                for n in range(start, start + j - 1):
                    actions.append(("advance", n))
                actions.append(("reverse", start + j))
            return
        m = _table(length, nfree)[1]
        for n in range(start, start + m):
            actions.append(("advance", n))
        sl = free.pop()
        actions.append(("store", sl, start + m))
        rev(start + m, length - m, sl, nfree - 1)
        actions.append(("free", sl))
        free.append(sl)
        actions.append(("restore", slot, start))
        rev(start, m, slot, nfree)

    rev(0, l, -1, s)
    return actions


def count_advances(actions) -> int:
    return sum(1 for a in actions if a[0] == "advance")


def binomial_closed_form(l: int, s: int) -> int:
    """Griewank-Walther's closed form of the minimal advance count.  Their
    snapshot count c includes the buffer holding x_0, so c = s + 1 here:
        T = r l - C(c + r, c + 1),  r = min{ r : C(c + r, c) >= l }."""
    from math import comb
    if l <= 1:
        return 0
    c = s + 1
    r = 0
    while comb(c + r, c) < l:
        r += 1
    return r * l - comb(c + r, c + 1)
