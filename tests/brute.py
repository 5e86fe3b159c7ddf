"""Brute-force enumeration of every global alignment of tiny pairs.

Independent of the oracle: no DP recurrence, just every path through the
alignment grid, each priced from the gap model (x per mismatch, o + L e per
maximal gap run of L bases), and a tie-break selector that works on the set
of optimal op strings rather than on DP values.
"""
from __future__ import annotations

import functools
import itertools

import numpy as np


@functools.lru_cache(maxsize=None)
def paths(m: int, n: int):
    """All move strings ('M' diagonal, 'I' P-only, 'D' T-only) from (0,0) to (m,n)."""
    if m == 0 and n == 0:
        return ("",)
    out = []
    if m > 0 and n > 0:
        out += [p + "M" for p in paths(m - 1, n - 1)]
    if m > 0:
        out += [p + "I" for p in paths(m - 1, n)]
    if n > 0:
        out += [p + "D" for p in paths(m, n - 1)]
    return tuple(out)


@functools.lru_cache(maxsize=None)
def _shape(m: int, n: int, o: int, e: int):
    """Per path: gap cost, and the 0/1 incidence of its diagonal cells."""
    ps = paths(m, n)
    gap = np.zeros(len(ps), np.int64)
    inc = np.zeros((len(ps), max(m * n, 1)), np.int64)
    for t, p in enumerate(ps):
        i = j = 0
        prev = None
        for mv in p:
            if mv == "M":
                inc[t, i * n + j] = 1
                i += 1
                j += 1
            elif mv == "I":
                gap[t] += e + (o if prev != "I" else 0)
                i += 1
            else:
                gap[t] += e + (o if prev != "D" else 0)
                j += 1
            prev = mv
    return ps, gap, inc


def optimal_alignments(P, T, pen):
    """(min cost, list of optimal op strings over '=XID')."""
    _, x, o, e = pen
    m, n = len(P), len(T)
    ps, gap, inc = _shape(m, n, o, e)
    if m and n:
        mm = (np.asarray(P)[:, None] != np.asarray(T)[None, :]).astype(np.int64).reshape(-1)
        cost = gap + x * (inc @ mm)
    else:
        cost = gap
    best = int(cost.min())
    out = []
    for t in np.nonzero(cost == best)[0]:
        i = j = 0
        s = []
        for mv in ps[t]:
            if mv == "M":
                s.append("=" if P[i] == T[j] else "X")
                i += 1
                j += 1
            elif mv == "I":
                s.append("I")
                i += 1
            else:
                s.append("D")
                j += 1
        out.append("".join(s))
    return best, out


ORDER = "XID="


def select_canonical(strings, gap_open: int) -> str:
    """Pick one optimal op string by walking from the end over the *set*.

    Free mode: keep the strings whose current (last unconsumed) op is the
    first present in the order X, I, D, =.  Inside a gap run (only when
    gap_open > 0): prefer ending the run -- keep the strings whose preceding
    op differs from the run's op (or that end there), choosing among those in
    the order X, I, D, =; if none does, continue the run.
    """
    cands = list(strings)
    pos = 0  # ops consumed from the end
    run = None  # current gap op when inside a run
    while True:
        live = [s for s in cands if len(s) > pos]
        if not live:
            break
        if run is None:
            ops = {s[len(s) - 1 - pos] for s in live}
            pick = next(c for c in ORDER if c in ops)
            cands = [s for s in live if s[len(s) - 1 - pos] == pick]
            pos += 1
            if pick in "ID" and gap_open > 0:
                run = pick
        else:
            # current op is the run op (already consumed); look at the next one
            ending = [s for s in cands if len(s) <= pos or s[len(s) - 1 - pos] != run]
            if ending:
                done = [s for s in ending if len(s) <= pos]
                if done:
                    cands = done
                    break
                ops = {s[len(s) - 1 - pos] for s in ending}
                pick = next(c for c in ORDER if c in ops)
                cands = [s for s in ending if s[len(s) - 1 - pos] == pick]
                pos += 1
                run = pick if (pick in "ID") else None
            else:
                pos += 1
    assert len(set(cands)) == 1, cands
    return cands[0]


def rle(s: str):
    return ["%d%s" % (len(list(g)), k) for k, g in itertools.groupby(s)]


def rle_string(s: str) -> str:
    return "".join(rle(s))
