"""Pins of the scalar wavefront oracle's work counters (CPU).

The counters are the algorithmic work of the wavefront algorithm (paper,
"Wavefront Algorithm (WFA)": O(n s) work, one unit per diagonal of every
wavefront): the WFA roofline divides them by kernel time, so they are pinned
here against values derived by hand from the recurrences' ranges, not against
the code that counts them:

* an identical pair is aligned at s = 0 by one extension: one cell, one
  wavefront, L bases compared, ceil(L / 32) words;
* an empty pattern against n bases (unit costs 1/0/1): every score s <= n has
  the range [0, min(s, n)] (the lower end is clipped at -m = 0, the upper end
  grows by one per score), so cells = (n + 1)(n + 2) / 2;
* the same under 4/6/2: only s = 0 and the even scores from 4 on are
  non-null, hi_s = s / 2 - 1 clipped at n, the optimum 6 + 2n ends the run,
  so cells = 1 + n(n + 1) / 2 + 3n + 2;
* two tiny cases worked out wavefront by wavefront (in the comments below).

A planted-mistake test compiles mutated copies of the oracle and checks that
these pins catch each mutation.
"""
import os
import shutil
import subprocess

import pytest

import oracle

PEN = (0, 4, 6, 2)


def counter_pins(handle=None):
    """Every pin; returns the list of failures (empty when all hold)."""
    bad = []

    def check(label, P, T, pen, want):
        st, sc, _, w = oracle.wfa_pair(P, T, pen, handle=handle)
        got = {k: w[k] for k in want if k in w}
        if "score" in want:
            got["score"] = sc
        if got != want:
            bad.append((label, got, want))

    for L in [0, 1, 5, 31, 32, 33, 64, 100]:
        s = ("ACGT" * 30)[:L]
        check("identical %d" % L, s, s, PEN,
              dict(score=0, cells=1, wavefronts=1, compared=L, words=(L + 31) // 32, lo_min=0, hi_max=0))
    for n in range(1, 16):
        T = ("GATTACA" * 4)[:n]
        check("empty pattern 1/0/1 n=%d" % n, "", T, (0, 1, 0, 1),
              dict(score=n, cells=(n + 1) * (n + 2) // 2, wavefronts=n + 1, compared=0, words=0,
                   lo_min=0, hi_max=n))
        check("empty pattern 4/6/2 n=%d" % n, "", T, PEN,
              dict(score=6 + 2 * n, cells=1 + n * (n + 1) // 2 + 3 * n + 2, compared=0, words=0,
                   lo_min=0, hi_max=n))
    # P = A, T = C under 4/6/2: s = 0 is one cell whose extension stops at
    # once on the mismatch (1 base compared, 1 word); s = 2 has no source
    # (the s = 0 wavefront has no I or D component); s = 4 takes M_0 through
    # a mismatch: range [-1, 1], M_4[0] = 1 reaches the end cell (its
    # extension stops at the end: 0 words).  cells 1 + 3.
    check("A vs C", "A", "C", PEN,
          dict(score=4, cells=4, wavefronts=2, compared=1, words=1, lo_min=-1, hi_max=1))
    # P = AAAA, T = AAAAC: s = 0 extends 4 matches to the end of P (4
    # compared, 1 word); s = 4: [-1, 1], every candidate out of the table;
    # s = 6: [-2, 2] from the (absent) I, D of s = 4; s = 8: [-3, 3], where
    # D_8[1] = M_0[0] + 1 = 5 is the end cell.  cells 1 + 3 + 5 + 7.
    check("AAAA vs AAAAC", "AAAA", "AAAAC", PEN,
          dict(score=8, cells=16, wavefronts=4, compared=4, words=1, lo_min=-3, hi_max=3))
    return bad


def test_wfa_work_counters_pinned():
    bad = counter_pins()
    assert not bad, bad[:3]


def test_wfa_work_counters_consistent_on_random_pairs():
    # compared >= words - wavefront extensions stopped at an end, words <=
    # compared + cells; both grow with the pair; cells >= wavefronts
    import numpy as np
    rng = np.random.default_rng(5)
    for _ in range(50):
        L = int(rng.integers(1, 300))
        T = rng.integers(0, 4, L).astype(np.uint8)
        P = T.copy()
        flip = rng.random(L) < 0.05
        P[flip] = (P[flip] + 1) % 4
        st, sc, _, w = oracle.wfa_pair(P, T, PEN)
        assert w["cells"] >= w["wavefronts"] >= 1
        assert w["words"] <= w["compared"] + w["cells"]
        assert w["compared"] >= L - int(flip.sum())  # the matching bases are compared at least once
        assert w["lo_min"] <= 0 <= w["hi_max"]


# (file, anchor, replacement): each must be caught by counter_pins
MUTANTS = [
    ("wfa_scalar.c", "lo -= 1; hi += 1;", "lo -= 1; hi += 2;"),       # width update
    ("wfa_scalar.c", "if (hi > n) hi = n;", ""),                       # upper clip dropped
    ("wfa_scalar.c", "      S.cells += 1;\n", "\n"),                   # s = 0 not counted
    ("wfa_scalar.c", "S.words += run / 32 + 1;", "S.words += run / 32;"),  # stop word lost
    ("wfa_scalar.c", "        S.compared += 1;\n", "\n"),              # mismatch not compared
    ("wfa_scalar.c", "S.cells += width;", "S.cells += width - 1;"),    # off by one per score
]


@pytest.mark.parametrize("idx", range(len(MUTANTS)))
def test_counter_pins_catch_planted_mistakes(tmp_path, idx):
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
    assert counter_pins(oracle.bind(so)), "planted mistake %d went unnoticed" % idx
