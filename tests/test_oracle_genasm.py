"""Pins of the GenASM oracle (oracle/genasm.c), CPU.

What pins it, apart from itself:
* its distance calculation against the textbook prefix edit-distance table
  (status bit [j, d, i] must be [D(i, j) <= d], anchored and free starts);
* with one window covering the pair, the score is the Levenshtein distance
  and the CIGAR replays both sequences at that many edits;
* hand-worked tracebacks (the gap-extension preference, the start row and
  column, a two-window pair);
* windowed runs on workload-shaped pairs: valid CIGARs, score = edits >=
  Levenshtein, 0 for identical pairs, 1 for a lone substitution;
* the threshold: accepted results do not depend on k, and k one below the
  score rejects;
* a second form of the same reading written on plain DP tables (no bit
  vectors) on many tiny pairs and window shapes;
* planted mistakes in a copy of the oracle must each fail one of these.
"""
import itertools
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from oracle import genasm_dc, genasm_pair, rescore, cigar_string

EDIT = (0, 1, 0, 1)


def _c(s):
    return np.array(["ACGT".index(ch) for ch in s], np.uint8)


def prefix_table(p, t, anchored):
    """D(i, j): fewest unit edits aligning p[:i] with t[:j]; the start row
    and column cost i (j) when anchored, 0 when free."""
    a, b = len(p), len(t)
    D = np.zeros((a + 1, b + 1), np.int64)
    for i in range(a + 1):
        D[i, 0] = i if anchored else 0
    for j in range(b + 1):
        D[0, j] = j if anchored else 0
    for i in range(1, a + 1):
        for j in range(1, b + 1):
            D[i, j] = min(D[i - 1, j - 1] + (p[i - 1] != t[j - 1]), D[i - 1, j] + 1, D[i, j - 1] + 1)
    return D


def lev(p, t):
    return int(prefix_table(p, t, True)[len(p), len(t)])


def _rand_pair(rng, m, rate):
    p = rng.integers(0, 4, m).astype(np.uint8)
    t = []
    for ch in p:
        u = rng.random()
        if u < rate / 3:
            t.append((int(ch) + 1 + rng.integers(0, 3)) % 4)
        elif u < 2 * rate / 3:
            continue
        elif u < rate:
            t.append(int(ch))
            t.append(int(rng.integers(0, 4)))
        else:
            t.append(int(ch))
    return p, np.array(t, np.uint8)


# ------------------------------------------------------------ distance calculation


@pytest.mark.parametrize("anchored", [True, False])
def test_status_bits_are_the_thresholded_prefix_table(anchored):
    rng = np.random.default_rng(11 + anchored)
    cases = [(rng.integers(0, 4, rng.integers(0, 10)).astype(np.uint8),
              rng.integers(0, 4, rng.integers(0, 10)).astype(np.uint8)) for _ in range(300)]
    cases += [(np.zeros(0, np.uint8), np.zeros(0, np.uint8)), (_c("ACGT"), _c("ACGT"))]
    for p, t in cases:
        L = max(len(p), len(t)) + 1
        R = genasm_dc(p, t, anchored, L)
        D = prefix_table(p, t, anchored)
        want = np.stack([[D[:, j] <= d for d in range(L + 1)] for j in range(len(t) + 1)]).astype(np.uint8)
        assert np.array_equal(R, want), (p, t, anchored)


# ------------------------------------------------------------ one window: exact


def test_one_window_is_levenshtein_exhaustive():
    seqs = [np.array(s, np.uint8) for n in range(5) for s in itertools.product(range(3), repeat=n)]
    for p in seqs:
        for t in seqs:
            st, sc, runs = genasm_pair(p, t, -1, window=8, overlap=0)
            assert st == 0
            assert sc == lev(p, t)
            assert rescore(p, t, runs, EDIT) == sc


def test_one_window_is_levenshtein_random():
    rng = np.random.default_rng(5)
    for _ in range(200):
        p, t = _rand_pair(rng, int(rng.integers(1, 60)), 0.2)
        st, sc, runs = genasm_pair(p, t, -1)  # 64-base window covers the pair
        assert (st, sc) == (0, lev(p, t))
        assert rescore(p, t, runs, EDIT) == sc


# ------------------------------------------------------------ hand-worked tracebacks


def test_gap_extension_first():
    # P = AAC, T = A.  From (3, 1) with budget 2: p3 = C != A and D(2, 0) = 2
    # > 1, so no match or substitution; insertion: D(2, 1) = 1 <= 1 -> 'I'.
    # At (2, 1), budget 1, previous 'I': insertion D(1, 1) = 0 <= 0 -> 'I'
    # again (a match, D(1, 0) = 1 <= 1, was also available and would come
    # next without the preference).  (1, 1): '='.  Forward: 1= 2I.
    assert genasm_pair(_c("AAC"), _c("A")) == (0, 2, [1 << 4 | 0, 2 << 4 | 2])
    # the mirror case gives deletions
    assert genasm_pair(_c("A"), _c("AAC")) == (0, 2, [1 << 4 | 0, 2 << 4 | 3])


def test_match_before_gap_without_a_run():
    # P = A, T = AA: from (1, 2) the match (D(0, 1) = 1 <= 1) comes before the
    # deletion, which the start row then forces: forward 1D 1=.
    assert genasm_pair(_c("A"), _c("AA")) == (0, 1, [1 << 4 | 3, 1 << 4 | 0])


def test_two_windows_by_hand():
    # W = 3, O = 1 (commit 2 bases).  P = ACGTA, T = ACTA.
    # Window 1 (free start): GTA against CTA, distance 1; the walk from (3, 3)
    # takes '=' (A/A, D(2, 2) = 1) and '=' (T/T, D(1, 1) = 1), has consumed 2
    # bases and stops: 3 pattern and 2 text bases remain.
    # Window 2 (final, anchored): ACG against AC, distance 1; 'I' for the G
    # (no match, D(2, 1) = 1 > 0 rules out 'X'), then '=' '='.
    # Forward: 2= 1I 2=, one edit.
    assert genasm_pair(_c("ACGTA"), _c("ACTA"), -1, window=3, overlap=1) == (0, 1, [2 << 4, 1 << 4 | 2, 2 << 4])


def test_empty_sides():
    assert genasm_pair(_c(""), _c("ACG")) == (0, 3, [3 << 4 | 3])
    assert genasm_pair(_c("ACG"), _c("")) == (0, 3, [3 << 4 | 2])
    assert genasm_pair(_c(""), _c("")) == (0, 0, [])
    assert genasm_pair(_c(""), _c("ACG"), 2) == (1, -1, [])
    assert genasm_pair(_c(""), _c("ACG"), 3)[0] == 0


# ------------------------------------------------------------ work counters


def test_work_counters():
    rng = np.random.default_rng(13)
    # identical 150-base pair: windows end at 150, 110, 70 (each commits 40
    # '=' ops) and the final one covers 30 bases; every distance is 0, so the
    # updates are 64 + 64 + 64 + 30
    p = rng.integers(0, 4, 150).astype(np.uint8)
    assert genasm_pair(p, p, stats=True)[3] == {"windows": 4, "updates": 222, "tb_steps": 150}
    # one window: (Levenshtein + 1) x n updates, one step per op
    for _ in range(30):
        a, b = _rand_pair(rng, int(rng.integers(1, 60)), 0.2)
        st, sc, runs, c = genasm_pair(a, b, stats=True)
        assert c == {"windows": 1, "updates": (lev(a, b) + 1) * len(b), "tb_steps": sum(r >> 4 for r in runs)}
    # an empty side aligns no window
    assert genasm_pair(_c(""), _c("ACG"), stats=True)[3] == {"windows": 0, "updates": 0, "tb_steps": 0}


# ------------------------------------------------------------ windowed pairs


def test_windowed_pairs_are_valid_alignments():
    rng = np.random.default_rng(7)
    for it in range(60):
        m = int(rng.integers(100, 400))
        p, t = _rand_pair(rng, m, float(rng.uniform(0, 0.12)))
        st, sc, runs = genasm_pair(p, t)
        assert st == 0
        assert rescore(p, t, runs, EDIT) == sc
        assert sc >= lev(p, t)


def test_identical_and_lone_substitution():
    rng = np.random.default_rng(8)
    for _ in range(20):
        p = rng.integers(0, 4, int(rng.integers(65, 500))).astype(np.uint8)
        assert genasm_pair(p, p) == (0, 0, [len(p) << 4])
        t = p.copy()
        q = int(rng.integers(0, len(p)))
        t[q] = (t[q] + 1) % 4
        st, sc, runs = genasm_pair(p, t)
        assert (st, sc) == (0, 1)
        assert cigar_string(runs) == "".join(
            s for s in ("%d=" % q if q else "", "1X", "%d=" % (len(p) - q - 1) if q < len(p) - 1 else ""))


def test_threshold():
    rng = np.random.default_rng(9)
    for _ in range(40):
        p, t = _rand_pair(rng, int(rng.integers(50, 300)), 0.1)
        st, sc, runs = genasm_pair(p, t, -1)
        assert st == 0
        assert genasm_pair(p, t, sc) == (0, sc, runs)
        assert genasm_pair(p, t, sc + 5) == (0, sc, runs)
        if sc > 0:
            assert genasm_pair(p, t, sc - 1) == (1, -1, [])


# ------------------------------------------------------------ the reading on DP tables


def genasm_by_tables(p, t, k, W, O):
    """The windowed reading again, on plain prefix tables (no bit vectors)."""
    C = W - O
    me, ne = len(p), len(t)
    ops, used, prev = [], 0, None
    while me > 0 and ne > 0:
        anchored = me <= W and ne <= W
        a, b = min(W, me), min(W, ne)
        pw, tw = p[me - a:me], t[ne - b:ne]
        D = prefix_table(pw, tw, anchored)
        cap = max(a, b) if k < 0 else min(k - used, max(a, b))
        d = int(D[a, b])
        if d > cap:
            return 1, -1, []
        i, j = a, b
        while True:
            if anchored:
                if i == 0 and j == 0:
                    break
            elif a - i >= C or b - j >= C or i == 0 or j == 0:
                break
            if i == 0:
                op = "D"
            elif j == 0:
                op = "I"
            else:
                mt = pw[i - 1] == tw[j - 1] and D[i - 1, j - 1] <= d
                sb = D[i - 1, j - 1] <= d - 1
                ins = D[i - 1, j] <= d - 1
                de = D[i, j - 1] <= d - 1
                if prev == "I" and ins:
                    op = "I"
                elif prev == "D" and de:
                    op = "D"
                elif mt:
                    op = "="
                elif sb:
                    op = "X"
                elif ins:
                    op = "I"
                else:
                    assert de
                    op = "D"
            if op != "=":
                d -= 1
                used += 1
            i -= op != "D"
            j -= op != "I"
            ops.append(op)
            prev = op
        me -= a - i
        ne -= b - j
    ops += ["I"] * me + ["D"] * ne
    used += me + ne
    if k >= 0 and used > k:
        return 1, -1, []
    fwd = ops[::-1]
    runs = []
    for op, g in itertools.groupby(fwd):
        runs.append(len(list(g)) << 4 | "=XID".index(op))
    return 0, used, runs


def test_bit_vectors_match_the_table_form():
    rng = np.random.default_rng(12)
    shapes = [(1, 0), (2, 0), (2, 1), (3, 1), (4, 2), (5, 1), (6, 3), (8, 4)]
    for it in range(1500):
        W, O = shapes[it % len(shapes)]
        m = int(rng.integers(0, 14))
        p, t = _rand_pair(rng, m, 0.3) if rng.random() < 0.7 else (
            rng.integers(0, 4, m).astype(np.uint8), rng.integers(0, 4, int(rng.integers(0, 14))).astype(np.uint8))
        k = int(rng.integers(-1, 8))
        assert genasm_pair(p, t, k, window=W, overlap=O) == genasm_by_tables(p, t, k, W, O), (p, t, k, W, O)


# ------------------------------------------------------------ planted mistakes

MUTANTS = {
    "substitution term dropped": ("sb = w->R[at(w, j - 1, d - 1, i - 1)];", "sb = 0;"),
    "insertion read from the old column": ("in = w->R[at(w, j, d - 1, i - 1)];",
                                           "in = w->R[at(w, j - 1, d - 1, i - 1)];"),
    "start row off by one": ("return anchored ? (uint8_t)(j <= d) : 1;", "return anchored ? (uint8_t)(j < d) : 1;"),
    "no gap-extension preference": ("if (prev == G_I && w.In[c]) op = G_I;", "if (0) op = G_I;"),
    "commit length off by one": ("const int32_t C = W - Ov;", "const int32_t C = W - Ov + 1;"),
    "free start taken as anchored": ("const int anchored = me <= W && ne <= W;", "const int anchored = 1;"),
    "updates without level 0": ("stats[1] += (int64_t)(d + 1) * b;", "stats[1] += (int64_t)d * b;"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistakes_fail(tmp_path, name):
    old, new = MUTANTS[name]
    src = open(os.path.join(oracle.HERE, "genasm.c")).read()
    assert src.count(old) == 1, "mutation anchor not found"
    for f in ("aim_oracle.c", "wfa_scalar.c"):
        shutil.copy(os.path.join(oracle.HERE, f), tmp_path / f)
    (tmp_path / "genasm.c").write_text(src.replace(old, new))
    so = str(tmp_path / "libmut.so")
    subprocess.run(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-pthread", "-o", so,
                    str(tmp_path / "aim_oracle.c"), str(tmp_path / "wfa_scalar.c"), str(tmp_path / "genasm.c")],
                   check=True)
    h = oracle.bind(so)
    caught = False
    try:
        ident = np.random.default_rng(13).integers(0, 4, 150).astype(np.uint8)
        if genasm_pair(_c("AAC"), _c("A"), handle=h) != (0, 2, [16, 34]):
            caught = True
        elif genasm_pair(ident, ident, handle=h, stats=True)[3] != {"windows": 4, "updates": 222, "tb_steps": 150}:
            caught = True
        elif genasm_pair(_c("ACGTA"), _c("ACTA"), -1, 3, 1, handle=h) != (0, 1, [32, 18, 32]):
            caught = True
        else:
            rng = np.random.default_rng(3)
            for it in range(400):
                W, O = [(2, 1), (3, 1), (4, 2), (8, 4), (64, 24)][it % 5]
                p, t = _rand_pair(rng, int(rng.integers(0, 14)), 0.3)
                if genasm_pair(p, t, -1, W, O, handle=h) != genasm_by_tables(p, t, -1, W, O):
                    caught = True
                    break
                L = max(len(p), len(t))
                D = prefix_table(p, t, True)
                want = [[(D[:, j] <= d).astype(np.uint8).tolist() for d in range(L + 1)] for j in range(len(t) + 1)]
                if genasm_dc(p, t, True, L, handle=h).tolist() != want:
                    caught = True
                    break
    except (RuntimeError, ValueError, AssertionError):
        caught = True
    assert caught, name
