"""Lower bound of the optimal alignment cost used by the exact pre-alignment
filter (test infrastructure, like the rest of ``oracle``).

Paper: Introduction, the third way to speed up alignment -- filter out
highly dissimilar pairs before the DP, without losing accuracy: a pair may
be dropped only when it provably cannot meet the threshold.

For penalties (0, x, o, e) (linear gaps: o = 0, e = g) and a pair P (m
bases), T (n bases), every alignment pays at least min(x, e) per edit (a
mismatch costs x, a gap base e on top of its run's opening), and at least
one opening o when m != n (some gap run must exist).  So with lev(P, T) the
Levenshtein distance (the fewest edits of any alignment):

    A = min(x, e) * lev(P, T) + (o if m != n else 0)
    B = o + e * |m - n|            if m != n, else 0
    lower(P, T) = max(A, B)  <=  the optimal cost.

A is taken only when the shorter sequence has at most REACH bases (the
bit-vectors); beyond that, lower = B.  A pair is rejected by the filter iff
lower > max_score.
"""
from __future__ import annotations

import numpy as np

REACH = 1024


def lower_bounds(batch, alg: str, pen, nthreads=None):
    """int32 lower bound per pair of a ``synth.PairBatch`` (see module doc)."""
    from . import align_batch
    _, x, o, e = pen
    if alg == "nw":
        o = 0
    m = batch.pat_len.astype(np.int64)
    n = batch.txt_len.astype(np.int64)
    # Levenshtein distance = linear-gap NW with unit costs (pinned against a
    # two-row textbook Levenshtein in tests/test_oracle.py)
    lev, _, _, _ = align_batch(batch, "nw", (0, 1, 0, 1), -1, want_cigar=False, nthreads=nthreads)
    lev = lev.astype(np.int64)
    diff = m != n
    a = min(x, e) * lev + np.where(diff, o, 0)
    b = np.where(diff, o + e * np.abs(m - n), 0)
    out = np.where(np.minimum(m, n) <= REACH, np.maximum(a, b), b)
    return out.astype(np.int32)
