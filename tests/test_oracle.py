"""Pins for the CPU oracle: each check comes from outside the oracle itself.

* hand-derived cases (costs worked out from the gap model by hand);
* exhaustive brute force over every alignment of tiny pairs, with a
  set-based tie-break selector (tests/brute.py), for the optimum and the CIGAR;
* special cases that reduce to other routines: Gotoh with gap_open 0 equals
  linear NW; NW with unit costs equals a two-row Levenshtein distance;
* a second algorithm: the scalar WFA must reach the same optimum and CIGAR;
* invariants: the CIGAR replays and rescores to the score; thresholds; bounds.
"""
import itertools
import os
import shutil
import subprocess

import numpy as np
import pytest

import brute
import oracle
import synth
from oracle import align_pair, cigar_string, rescore, wfa_pair

AFFINE_PENS = [(0, 4, 6, 2), (0, 3, 4, 1), (0, 2, 1, 1), (0, 4, 2, 2), (0, 1, 3, 1), (0, 9, 1, 1)]
LINEAR_PENS = [(0, 1, 0, 1), (0, 3, 0, 4), (0, 2, 0, 1), (0, 5, 0, 1), (0, 3, 0, 1)]


def _all_seqs(alphabet, maxlen):
    for L in range(maxlen + 1):
        for s in itertools.product(alphabet, repeat=L):
            yield np.array(s, np.uint8)


# ---------------------------------------------------------------- hand cases

@pytest.mark.parametrize("alg,pen", [("nw", (0, 1, 0, 1)), ("swg", (0, 4, 6, 2)), ("wfa", (0, 4, 6, 2)),
                                     ("nw", (0, 3, 0, 4)), ("swg", (0, 3, 4, 1))])
def test_hand_cases(alg, pen):
    _, x, o, e = pen
    # identical sequences: cost 0, all matches
    assert align_pair("ACGTACGT", "ACGTACGT", alg, pen) == (0, 0, [(8 << 4) | 0])
    # one substitution in the middle: x, "3=1X3="
    st, sc, r = align_pair("ACGTACG", "ACGAACG", alg, pen)
    assert sc == min(x, 2 * (o + e)) and st == 0
    if x < 2 * (o + e):
        assert cigar_string(r) == "3=1X3="
    # one extra base in P: a single I run of length 1 costs o + e
    st, sc, r = align_pair("ACGTTACG", "ACGTACG", alg, pen)
    assert sc == o + e
    # the extra T can sit at P[3] or P[4]; the walk from the end places the
    # gap at the last feasible position, P[4]
    assert cigar_string(r) == "4=1I3="
    # one missing base in P: a single D
    st, sc, r = align_pair("ACGACG", "ACGTACG", alg, pen)
    assert sc == o + e and cigar_string(r) == "3=1D3="
    # empty pattern: one D run over the whole text
    assert align_pair("", "ACG", alg, pen) == (0, o + 3 * e, [(3 << 4) | 3])
    # empty text: one I run over the whole pattern
    assert align_pair("ACGT", "", alg, pen) == (0, o + 4 * e, [(4 << 4) | 2])
    # both empty
    assert align_pair("", "", alg, pen) == (0, 0, [])


def test_hand_affine_prefers_one_long_gap():
    # With o = 6, e = 2 a 2-base gap (10) beats two 1-base gaps (16) and two
    # mismatches of 4 each (8) beat a 2-base gap plus... here P drops "TT".
    st, sc, r = align_pair("ACGAAA", "ACGTTAAA", "swg", (0, 4, 6, 2))
    assert sc == 10 and cigar_string(r) == "3=2D3="
    # linear NW with g = 1 prices the same gap as 2
    st, sc, r = align_pair("ACGAAA", "ACGTTAAA", "nw", (0, 1, 0, 1))
    assert sc == 2


# ---------------------------------------------------------------- brute force

def _check_exhaustive(alphabet, maxlen, algs_pens):
    seqs = list(_all_seqs(alphabet, maxlen))
    bad = []
    for P in seqs:
        for T in seqs:
            for alg, pen in algs_pens:
                best, strings = brute.optimal_alignments(P, T, pen)
                st, sc, r = align_pair(P, T, alg, pen)
                canon = brute.rle_string(brute.select_canonical(strings, pen[2]))
                if sc != best or cigar_string(r) != canon:
                    bad.append((P.tolist(), T.tolist(), alg, pen, sc, best, cigar_string(r), canon))
    return bad


def test_exhaustive_acgt_len3():
    cases = [("swg", p) for p in AFFINE_PENS[:3] + AFFINE_PENS[-1:]] + [("nw", p) for p in LINEAR_PENS[:3]]
    bad = _check_exhaustive(range(4), 3, cases)
    assert not bad, bad[:5]


def test_exhaustive_binary_len5():
    cases = [("swg", p) for p in AFFINE_PENS] + [("nw", p) for p in LINEAR_PENS]
    bad = _check_exhaustive(range(2), 5, cases)
    assert not bad, bad[:5]


def test_exhaustive_wfa_matches_brute_force():
    seqs = list(_all_seqs(range(2), 4))
    for P in seqs:
        for T in seqs:
            for pen in AFFINE_PENS + [(0, 2, 0, 1)]:
                best, strings = brute.optimal_alignments(P, T, pen)
                st, sc, r, _ = wfa_pair(P, T, pen)
                assert sc == best
                assert cigar_string(r) == brute.rle_string(brute.select_canonical(strings, pen[2]))


# ---------------------------------------------------------------- special cases

def _lev(a, b):
    """Two-row Levenshtein distance (independent textbook routine)."""
    prev = list(range(len(b) + 1))
    for i in range(1, len(a) + 1):
        cur = [i] + [0] * len(b)
        for j in range(1, len(b) + 1):
            cur[j] = min(prev[j] + 1, cur[j - 1] + 1, prev[j - 1] + (a[i - 1] != b[j - 1]))
        prev = cur
    return prev[-1]


def _random_pairs(seed, count, maxlen, rate=0.1):
    rng = np.random.default_rng(seed)
    for _ in range(count):
        n = int(rng.integers(0, maxlen + 1))
        T = rng.integers(0, 4, n).astype(np.uint8)
        b = synth.from_lists([T], [T])
        pat, po = synth.mutate(rng, b.txt, b.txt_off, [rate if rng.random() < 0.8 else 0.5])
        yield pat, T


def test_nw_unit_costs_is_levenshtein():
    for P, T in _random_pairs(11, 300, 60, 0.15):
        st, sc, r = align_pair(P, T, "nw", (0, 1, 0, 1))
        assert sc == _lev(P.tolist(), T.tolist())


def test_gotoh_with_zero_open_equals_linear_nw():
    for P, T in _random_pairs(12, 300, 60, 0.15):
        for x, g in [(1, 1), (3, 4), (2, 1), (5, 1)]:
            a = align_pair(P, T, "nw", (0, x, 0, g))
            b = align_pair(P, T, "swg", (0, x, 0, g))
            assert a == b


def test_wfa_equals_gotoh_random():
    for P, T in _random_pairs(13, 300, 200, 0.06):
        for pen in [(0, 4, 6, 2), (0, 3, 4, 1)]:
            g = align_pair(P, T, "swg", pen)
            w = wfa_pair(P, T, pen)
            assert g == w[:3]


def test_wfa_equals_gotoh_long():
    for P, T in _random_pairs(14, 6, 1500, 0.05):
        g = align_pair(P, T, "swg", (0, 4, 6, 2))
        w = wfa_pair(P, T, (0, 4, 6, 2))
        assert g == w[:3]


def test_common_divisor_of_penalties():
    # Every alignment cost is a combination of x, o and e with non-negative
    # integer counts, so with g = gcd(x, o, e) the Gotoh optimum under
    # (x/g, o/g, e/g) is the optimum under (x, o, e) divided by g, reached by
    # the same canonical CIGAR (each comparison of the tie order scales by
    # g), and a threshold S_max becomes floor(S_max / g).  The GPU wavefront
    # kernels rely on this; here it is checked on the full-matrix oracle.
    for P, T in _random_pairs(21, 200, 120, 0.08):
        for pen, g in [((0, 4, 6, 2), 2), ((0, 40, 10, 30), 10), ((0, 6, 0, 3), 3)]:
            red = (0, pen[1] // g, pen[2] // g, pen[3] // g)
            alg = "nw" if pen[2] == 0 else "swg"
            st, sc, r = align_pair(P, T, alg, pen)
            st2, sc2, r2 = align_pair(P, T, alg, red)
            assert (st2, sc2 * g, r2) == (st, sc, r)
            for smax in [sc - 1, sc, sc + 1, sc + g]:
                if smax < 0:
                    continue
                got = align_pair(P, T, alg, red, max_score=smax // g)
                want = align_pair(P, T, alg, pen, max_score=smax)
                assert (got[0], got[1] * g if got[1] >= 0 else -1, got[2]) == want


# ---------------------------------------------------------------- invariants

def test_rescore_and_bounds_random():
    for P, T in _random_pairs(15, 400, 120, 0.1):
        m, n = len(P), len(T)
        for alg, pen in [("nw", (0, 1, 0, 1)), ("swg", (0, 4, 6, 2)), ("nw", (0, 3, 0, 4))]:
            _, x, o, e = pen
            st, sc, r = align_pair(P, T, alg, pen)
            assert rescore(P, T, r, pen) == sc
            gap = lambda L: (o + L * e) if L else 0
            assert sc <= gap(m) + gap(n)
            if m != n:
                assert sc >= o + abs(m - n) * e
            if np.array_equal(P, T):
                assert sc == 0


def test_threshold_semantics():
    for P, T in _random_pairs(16, 200, 80, 0.1):
        for alg, pen in [("nw", (0, 1, 0, 1)), ("swg", (0, 4, 6, 2)), ("wfa", (0, 4, 6, 2))]:
            full = align_pair(P, T, alg, pen)
            for smax in [0, 3, 8, 20, 60, 10_000]:
                st, sc, r = align_pair(P, T, alg, pen, max_score=smax)
                if full[1] <= smax:
                    assert (st, sc, r) == full
                else:
                    assert (st, sc, r) == (oracle.REJECTED, -1, [])
                if alg == "wfa":
                    w = wfa_pair(P, T, pen, max_score=smax)
                    assert w[:3] == (st, sc, r)


def test_batch_driver_matches_pairwise():
    b = synth.workload("nw100", n=300)
    score, status, cigar, off = oracle.align_batch(b, "nw", (0, 1, 0, 1), 5, nthreads=4)
    rej = 0
    for i in range(b.n):
        st, sc, r = align_pair(b.pattern(i), b.text(i), "nw", (0, 1, 0, 1), 5)
        assert (status[i], score[i]) == (st, sc)
        assert cigar[off[i]:off[i + 1]].tolist() == r
        rej += st == oracle.REJECTED
    assert 0 < rej < 30  # about 1.7 % of pairs exceed 5 edits at 2 % error


@pytest.mark.parametrize("name,count", [("swg150", 60), ("wfa250", 60), ("wfa_mixed", 6)])
def test_workload_samples_wfa_and_rescore(name, count):
    w = synth.WORKLOADS[name]
    b = synth.workload(name, n=count)
    for i in range(b.n):
        P, T = b.pattern(i), b.text(i)
        if len(T) > 3000:
            continue
        g = align_pair(P, T, "swg", w["pen"], w["max_score"])
        if g[0] == 0:
            assert rescore(P, T, g[2], w["pen"]) == g[1]
        wf = wfa_pair(P, T, w["pen"], w["max_score"])
        assert wf[:3] == g


# ---------------------------------------------------------------- planted mistakes

MUTANTS = [
    # dropped term: gap opening missing from the E recurrence
    ("aim_oracle.c", "AT(E, i, j) = min2(AT(H, i - 1, j) + o + e,", "AT(E, i, j) = min2(AT(H, i - 1, j) + e,"),
    # wrong index: F extends from the row above instead of the column to the left
    ("aim_oracle.c", "AT(F, i, j) = min2(AT(H, i, j - 1) + o + e, AT(F, i, j - 1) + e);",
     "AT(F, i, j) = min2(AT(H, i, j - 1) + o + e, AT(F, i - 1, j) + e);"),
    # wrong sign: match/mismatch cost inverted in NW
    ("aim_oracle.c", "int32_t c = P[i - 1] == T[j - 1] ? 0 : x;\n      AT(H, i, j) = min2(AT(H, i - 1, j - 1) + c, min2(AT(H, i - 1, j) + g",
     "int32_t c = P[i - 1] != T[j - 1] ? 0 : x;\n      AT(H, i, j) = min2(AT(H, i - 1, j - 1) + c, min2(AT(H, i - 1, j) + g"),
    # border: gap open dropped from the first column
    ("aim_oracle.c", "AT(H, i, 0) = AT(E, i, 0) = o + i * e;", "AT(H, i, 0) = AT(E, i, 0) = i * e;"),
    # tie-break: D tried before I in the Gotoh walk
    ("aim_oracle.c", "else if (i > 0 && h == AT(E, i, j)) state = 1;\n        else if (j > 0 && h == AT(F, i, j)) state = 2;",
     "else if (j > 0 && h == AT(F, i, j)) state = 2;\n        else if (i > 0 && h == AT(E, i, j)) state = 1;"),
    # tie-break: '=' tried before 'X'-free gaps in NW
    ("aim_oracle.c", "else if (i > 0 && h == AT(H, i - 1, j) + g) { rev[k++] = OP_I; --i; }",
     "else if (i > 0 && j > 0 && !mism && h == AT(H, i - 1, j - 1)) { rev[k++] = OP_EQ; --i; --j; }\n      else if (i > 0 && h == AT(H, i - 1, j) + g) { rev[k++] = OP_I; --i; }"),
    # tie-break: extend preferred over open when closing an I run
    ("aim_oracle.c", "if (AT(E, i, j) == AT(H, i - 1, j) + o + e) state = 0;\n        else if (i < 2 || AT(E, i, j) != AT(E, i - 1, j) + e) { rc = -2; break; }",
     "if (i >= 2 && AT(E, i, j) == AT(E, i - 1, j) + e) { }\n        else if (AT(E, i, j) == AT(H, i - 1, j) + o + e) state = 0;\n        else { rc = -2; break; }"),
]


@pytest.mark.parametrize("idx", range(len(MUTANTS)))
def test_pins_catch_planted_mistakes(tmp_path, idx):
    fname, old, new = MUTANTS[idx]
    src = open(os.path.join(oracle.HERE, fname)).read()
    assert src.count(old) == 1, "mutation anchor not found"
    for f in ("aim_oracle.c", "wfa_scalar.c", "genasm.c"):
        shutil.copy(os.path.join(oracle.HERE, f), tmp_path / f)
    (tmp_path / fname).write_text(src.replace(old, new))
    so = str(tmp_path / "libmut.so")
    subprocess.run(["gcc", "-O1", "-fPIC", "-shared", "-pthread", "-o", so,
                    str(tmp_path / "aim_oracle.c"), str(tmp_path / "wfa_scalar.c"),
                    str(tmp_path / "genasm.c")], check=True)
    h = oracle.bind(so)
    caught = False
    seqs = list(_all_seqs(range(2), 4))
    for P in seqs:
        for T in seqs:
            for alg, pen in [("swg", (0, 4, 6, 2)), ("swg", (0, 2, 1, 1)), ("swg", (0, 9, 1, 1)),
                             ("nw", (0, 2, 0, 1)), ("nw", (0, 1, 0, 1)), ("nw", (0, 3, 0, 1))]:
                best, strings = brute.optimal_alignments(P, T, pen)
                try:
                    st, sc, r = align_pair(P, T, alg, pen, handle=h)
                except RuntimeError:
                    caught = True
                    break
                canon = brute.rle_string(brute.select_canonical(strings, pen[2]))
                if sc != best or cigar_string(r) != canon:
                    caught = True
                    break
            if caught:
                break
        if caught:
            break
    assert caught, "planted mistake %d went unnoticed" % idx
