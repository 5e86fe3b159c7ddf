"""Pins of the WFA-adaptive oracle (oracle/wfa_scalar.c, its reduction
step), CPU.

The reduction is a heuristic, so the pins are: a hand-worked trace of the
drop rule (which diagonals go, when, and what that leaves), a hand-built pair
on which dropping loses the optimum, validity of every adaptive alignment
(its CIGAR replays both sequences at the score it reports) with a cost never
below the optimum, and identity with exact WFA whenever the rule cannot
fire.  Planted mistakes in a copy of the oracle (the distance taken as the
smaller remaining length, the reduction before the extension, a strict
threshold, the range test ignored) must each fail one of them.
"""
import os
import subprocess

import numpy as np
import pytest

import oracle
import synth

EDIT = (0, 1, 0, 1)


def _codes(s):
    return np.frombuffer(s.encode(), np.uint8).copy()


def _hand_case(handle=None, adaptive=(2, 0)):
    # P = CAAAAAAA, T = AAAAAAAG, edit costs.  s = 0: M[0] = 0 (C/A).  s = 1:
    # k = -1 (I) extends 7 to f = 7 (i = 8), k = 0 (X) extends 6 to f = 7,
    # k = 1 (D) stops at f = 1.  Distances max(m - i, n - f): 1, 1, 8; with
    # max_dist 0 diagonal 1 goes.  s = 2: M[0] = max(X 8, D from M[-1] 8) = 8
    # = n, the end: score 2, cells 1 + 3 + 4 (range [-2, 1]), 1 dropped.
    return oracle.wfa_pair(_codes("CAAAAAAA"), _codes("AAAAAAAG"), EDIT, handle=handle, adaptive=adaptive)


def test_hand_trace():
    st, sc, runs, c = _hand_case()
    assert (st, sc) == (0, 2)
    assert c["dropped"] == 1 and c["cells"] == 8
    assert oracle.cigar_string(runs) == "1X6=1X"
    # exact: the same optimum, one more cell at s = 2 (range [-2, 2])
    st, sc, runs2, c2 = oracle.wfa_pair(_codes("CAAAAAAA"), _codes("AAAAAAAG"), EDIT)
    assert (st, sc, runs2) == (0, 2, runs) and c2["cells"] == 9 and c2["dropped"] == 0
    # below min_len nothing is dropped: widths are 1, 3, 5
    st, sc, runs3, c3 = _hand_case(adaptive=(4, 0))
    assert c3["dropped"] == 0 and c3["cells"] == 9 and runs3 == runs


def test_dropping_loses_the_optimum():
    # P = GG + S, T = S + GG (S = ACGTACGTAC): the optimum (4 edits) opens
    # with two I.  At s = 1 the distances are 12, 11, 12 on diagonals -1, 0,
    # 1, so max_dist 0 removes -1 and with it the only way to reach -2 at
    # s = 2; the heuristic ends above the optimum.  A loose threshold keeps
    # every diagonal with an offset (it still trims absent ones at the ends,
    # which changes nothing) and finds the optimum.
    P, T = _codes("GGACGTACGTAC"), _codes("ACGTACGTACGG")
    ex = oracle.wfa_pair(P, T, EDIT)
    assert ex[:2] == (0, 4)
    tight = oracle.wfa_pair(P, T, EDIT, adaptive=(1, 0))
    assert tight[0] == 0 and tight[1] > 4 and tight[3]["dropped"] > 0
    assert oracle.rescore(P, T, tight[2], EDIT) == tight[1]
    loose = oracle.wfa_pair(P, T, EDIT, adaptive=(1, 1000))
    assert loose[:3] == ex[:3]


def _random_pairs(seed, n, lmax, rate_max):
    rng = np.random.default_rng(seed)
    pats, txts = [], []
    for _ in range(n):
        T = rng.integers(0, 4, int(rng.integers(0, lmax + 1))).astype(np.uint8)
        bb = synth.from_lists([T], [T])
        P, _ = synth.mutate(rng, bb.txt, bb.txt_off, [float(rng.uniform(0, rate_max))])
        pats.append(P)
        txts.append(T)
    return synth.from_lists(pats, txts)


@pytest.mark.parametrize("pen", [(0, 4, 6, 2), EDIT, (0, 3, 4, 1), (0, 9, 1, 1)])
def test_valid_and_never_below_optimum(pen):
    # The score is the wavefront score that reached the end.  The walk spends
    # it exactly, one open per gap step taken from M; when two such opens of
    # one gap type are adjacent (possible only once the cheaper extension was
    # dropped), the CIGAR merges them into one run and costs o less.  So:
    # optimum <= cost(CIGAR) <= score, and equality unless the rule fired.
    b = _random_pairs(5, 120, 300, 0.25)
    opt = oracle.align_batch(b, "swg" if pen[2] else "nw", pen, -1, want_cigar=False)[0]
    fired = 0
    for adaptive in [(10, 50), (4, 5), (1, 0)]:
        sc, st, cg, off = oracle.wfa_batch(b, pen, -1, adaptive=adaptive)
        assert (st == 0).all() and (sc >= opt).all()
        for i in range(b.n):
            cost = oracle.rescore(b.pattern(i), b.text(i), cg[off[i]:off[i + 1]], pen)
            assert opt[i] <= cost <= sc[i]
            if sc[i] == opt[i]:
                assert cost == sc[i]
        fired += int((sc > opt).sum())
    assert fired > 0  # the heuristic does lose the optimum on some pairs


def test_exact_when_the_rule_cannot_fire():
    b = _random_pairs(6, 200, 300, 0.2)
    pen = (0, 4, 6, 2)
    ex = oracle.wfa_batch(b, pen)
    # no wavefront reaches 2 * 300 + 2 diagonals, and no distance gap passes 10^6
    for adaptive in [(2 * 300 + 2, 0), (1, 10 ** 6)]:
        got = oracle.wfa_batch(b, pen, adaptive=adaptive)
        for a, c in zip(got, ex):
            assert np.array_equal(a, c)


def test_threshold_rejects_like_exact():
    b = _random_pairs(7, 200, 200, 0.3)
    pen = (0, 4, 6, 2)
    sc, st, _, _ = oracle.wfa_batch(b, pen, -1, adaptive=(10, 50))
    sc2, st2, _, off2 = oracle.wfa_batch(b, pen, 60, adaptive=(10, 50))
    assert np.array_equal(st2, np.where(sc > 60, 1, 0).astype(np.int8))
    assert np.array_equal(sc2, np.where(sc > 60, -1, sc))


MUTANTS = {
    "distance as the smaller remaining length":
        ("int32_t d = max2(m - (f - k), n - f);", "int32_t d = -max2(-(m - (f - k)), -(n - f));"),
    "strict threshold": ("- dmin <= max_dist) break;", "- dmin < max_dist) break;"),
    "range test ignored": ("if (min_len > 0 && w->hi - w->lo + 1 >= min_len) {", "if (min_len > 0) {"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistakes_fail(tmp_path, name):
    src = open(os.path.join(os.path.dirname(oracle.__file__), "wfa_scalar.c")).read()
    a, b = MUTANTS[name]
    n_sub = src.count(a)
    assert n_sub >= 1
    bad = src.replace(a, b)
    (tmp_path / "wfa_scalar.c").write_text(bad)
    so = str(tmp_path / "libmut.so")
    subprocess.run(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-pthread", "-o", so,
                    os.path.join(os.path.dirname(oracle.__file__), "aim_oracle.c"),
                    str(tmp_path / "wfa_scalar.c"),
                    os.path.join(os.path.dirname(oracle.__file__), "genasm.c")], check=True)
    h = oracle.bind(so)
    caught = False
    try:
        st, sc, runs, c = _hand_case(handle=h)
        if (st, sc, c["dropped"], c["cells"]) != (0, 2, 1, 8):
            caught = True
        st3 = _hand_case(handle=h, adaptive=(4, 0))[3]
        if st3["dropped"] != 0:
            caught = True
    except Exception:
        caught = True
    assert caught, name
