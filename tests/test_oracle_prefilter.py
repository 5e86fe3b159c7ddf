"""Pins of the pre-alignment lower bound (oracle/prefilter.py), CPU.

The bound must never exceed the optimal cost (soundness: the filter may
only drop pairs that cannot meet a threshold), checked exhaustively on
tiny pairs and on random pairs under several penalty sets against the
full-matrix oracle; it must be tight where the mathematics says so (a
single mismatch with x <= e, a single gap base with o = 0, identical pairs,
a pure length difference); and its Levenshtein term must equal an
independent two-row Levenshtein.
"""
import itertools

import numpy as np

import oracle
import synth
from oracle.prefilter import REACH, lower_bounds

PENS = [("swg", (0, 4, 6, 2)), ("swg", (0, 3, 4, 1)), ("nw", (0, 1, 0, 1)), ("nw", (0, 3, 0, 4)),
        ("swg", (0, 9, 1, 1)), ("swg", (0, 1, 5, 3)), ("wfa", (0, 4, 6, 2))]


def _lev(a, b):
    prev = list(range(len(b) + 1))
    for i in range(1, len(a) + 1):
        cur = [i] + [0] * len(b)
        for j in range(1, len(b) + 1):
            cur[j] = min(prev[j] + 1, cur[j - 1] + 1, prev[j - 1] + (a[i - 1] != b[j - 1]))
        prev = cur
    return prev[-1]


def _optimum(batch, alg, pen):
    return oracle.align_batch(batch, "nw" if alg == "nw" else "swg", pen, -1, want_cigar=False)[0]


def test_sound_exhaustive_tiny():
    seqs = [np.array(s, np.uint8) for L in range(4) for s in itertools.product(range(4), repeat=L)]
    pats, txts = zip(*[(p, t) for p in seqs for t in seqs])
    b = synth.from_lists(list(pats), list(txts))
    for alg, pen in PENS:
        lb = lower_bounds(b, alg, pen)
        assert (lb <= _optimum(b, alg, pen)).all(), (alg, pen)


def test_sound_random_and_levenshtein_term():
    rng = np.random.default_rng(3)
    pats, txts = [], []
    for _ in range(400):
        L = int(rng.integers(0, 120))
        T = rng.integers(0, 4, L).astype(np.uint8)
        if rng.random() < 0.3:
            P = rng.integers(0, 4, int(rng.integers(0, 120))).astype(np.uint8)  # unrelated
        else:
            bb = synth.from_lists([T], [T])
            P, _ = synth.mutate(rng, bb.txt, bb.txt_off, [float(rng.uniform(0, 0.3))])
        pats.append(P)
        txts.append(T)
    b = synth.from_lists(pats, txts)
    for alg, pen in PENS:
        lb = lower_bounds(b, alg, pen)
        assert (lb <= _optimum(b, alg, pen)).all(), (alg, pen)
    # the Levenshtein term against the textbook routine (x = e = 1, o = 0)
    lb = lower_bounds(b, "nw", (0, 1, 0, 1))
    want = [_lev(b.pattern(i).tolist(), b.text(i).tolist()) for i in range(b.n)]
    assert lb.tolist() == want


def test_tight_cases():
    b = synth.from_lists(["ACGT", "ACGT", "ACGT", "AAAA", "", "ACGTAC"],
                         ["ACGT", "AGGT", "ACT", "AAAAAAA", "ACG", "ACGTAC"])
    # identical: 0; one mismatch with x <= e: x; one deletion with o = 0: e
    assert lower_bounds(b, "swg", (0, 2, 0, 3)).tolist()[:2] == [0, 2]
    assert lower_bounds(b, "nw", (0, 4, 0, 3)).tolist()[2] == 3
    # a pure length difference: o + e * |m - n|, exactly the optimum
    lb = lower_bounds(b, "swg", (0, 4, 6, 2))
    opt = _optimum(b, "swg", (0, 4, 6, 2))
    assert lb[3] == opt[3] == 6 + 2 * 3 and lb[4] == opt[4] == 6 + 2 * 3 and lb[5] == 0


def test_reach():
    # a pattern longer than the bit-vectors reach keeps only the length term
    rng = np.random.default_rng(9)
    T = rng.integers(0, 4, REACH + 10).astype(np.uint8)
    P = rng.integers(0, 4, REACH + 5).astype(np.uint8)
    b = synth.from_lists([P, P[:REACH]], [T, T[:REACH + 3]])
    lb = lower_bounds(b, "swg", (0, 4, 6, 2))
    assert lb[0] == 6 + 2 * 5
    assert lb[1] > 6 + 2 * 3  # within reach: the Levenshtein term of unrelated sequences
