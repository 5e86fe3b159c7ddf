"""CIGAR validity check by replay (test infrastructure).

Replays an RLE CIGAR over the pattern P and text T and recomputes its cost
straight from the gap model of the paper's algorithms (System and Methods:
NW with a per-base gap cost, SWG/WFA with gap open + extend): '=' must pair
equal bases, 'X' unequal ones, 'I' consumes a base of P only, 'D' a base of T
only, the ops must consume P and T exactly, and the cost is the sum of x per
'X' plus o + L e per maximal run of L 'I' (or 'D').  No DP is involved, so it
checks any aligner's output independently.
"""
from __future__ import annotations

OPS = "=XID"


def parse_runs(runs):
    """uint32 runs (len << 4 | op) -> list of (op char, length)."""
    out = []
    for r in runs:
        r = int(r)
        op = r & 15
        if op > 3:
            raise ValueError("bad op code %d" % op)
        out.append((OPS[op], r >> 4))
    return out


def cigar_string(runs) -> str:
    return "".join("%d%s" % (n, op) for op, n in parse_runs(runs))


def rescore(P, T, runs, pen) -> int:
    """Return the cost of the alignment ``runs`` of P against T; raise
    ValueError if the CIGAR is not a valid alignment of the two sequences."""
    _, x, o, e = pen
    i = j = 0
    cost = 0
    prev = None
    for op, n in parse_runs(runs):
        if n <= 0:
            raise ValueError("empty run")
        if op == prev:
            raise ValueError("adjacent runs with the same op")
        prev = op
        if op in "=X":
            if i + n > len(P) or j + n > len(T):
                raise ValueError("CIGAR runs past a sequence end")
            for t in range(n):
                eq = int(P[i + t]) == int(T[j + t])
                if (op == "=") != eq:
                    raise ValueError("op %s at P[%d], T[%d] disagrees with the bases" % (op, i + t, j + t))
            if op == "X":
                cost += n * x
            i += n
            j += n
        elif op == "I":
            if i + n > len(P):
                raise ValueError("I run past the end of P")
            cost += o + n * e
            i += n
        else:
            if j + n > len(T):
                raise ValueError("D run past the end of T")
            cost += o + n * e
            j += n
    if i != len(P) or j != len(T):
        raise ValueError("CIGAR consumes (%d, %d) of (%d, %d)" % (i, j, len(P), len(T)))
    return cost
