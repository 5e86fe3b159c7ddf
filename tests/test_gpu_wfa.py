"""Bit-exact parity of the GPU wavefront kernels against the CPU oracle.

The oracle of the WFA path is the Gotoh definition (the wavefront algorithm
reaches the same optimum and, with the canonical tie order, the same CIGAR);
pairs too long for the full-matrix oracle's memory are checked against the
scalar WFA, which the CPU tests pin to Gotoh.
"""
import itertools

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
import synth  # noqa: E402
import paper_2208_01243_amd as aim  # noqa: E402
from gpu_util import compare, describe, run  # noqa: E402

AFF = (0, 4, 6, 2)


@pytest.fixture(scope="module")
def ctx():
    c = aim.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def ctx_plain():
    c = aim.Context(0, kernel="plain")
    yield c
    c.close()


def check(ctx, batch, pen=AFF, max_score=-1, **kw):
    got = run(ctx, batch, "wfa", pen, max_score, **kw)
    want = oracle.align_batch(batch, "wfa", pen, max_score)
    bad = compare(got, want)
    assert not bad, "%d mismatches, first: %s" % (len(bad), describe(batch, bad[0], got, want))
    return got


def _tiny_all(alphabet, maxlen):
    seqs = [np.array(s, np.uint8) for L in range(maxlen + 1) for s in itertools.product(alphabet, repeat=L)]
    pats, txts = zip(*[(p, t) for p in seqs for t in seqs])
    return synth.from_lists(list(pats), list(txts))


@pytest.mark.parametrize("pen", [AFF, (0, 3, 4, 1), (0, 2, 1, 1), (0, 9, 1, 1), (0, 1, 0, 1), (0, 5, 0, 2),
                                 (0, 40, 10, 30), (0, 41, 10, 29)])
# (0, 40, 10, 30) runs as (4, 1, 3) with scores times 10; (0, 41, 10, 29) has
# a ring of 42 scores, beyond the one-wavefront pass
def test_exhaustive_tiny(ctx, pen):
    check(ctx, _tiny_all(range(4), 3), pen)


def test_exhaustive_tiny_binary(ctx):
    b = _tiny_all(range(2), 5)
    for pen in [AFF, (0, 2, 1, 1)]:
        check(ctx, b, pen)
        check(ctx, b, pen, max_score=6)


def test_wfa250_first_20k(ctx):
    w = synth.WORKLOADS["wfa250"]
    b = synth.workload("wfa250", n=20_000)
    got = check(ctx, b, w["pen"], w["max_score"])
    rej = (got[1] == aim.PAIR_REJECTED).mean()
    assert 0.15 < rej < 0.25  # the unrelated fifth of the pairs


def test_plain_equals_oracle(ctx_plain):
    w = synth.WORKLOADS["wfa250"]
    check(ctx_plain, synth.workload("wfa250", n=2000), w["pen"], w["max_score"])


def _mixed(seed, count, lmin, lmax, rates):
    rng = np.random.default_rng(seed)
    pats, txts = [], []
    for _ in range(count):
        L = int(rng.integers(lmin, lmax + 1))
        T = rng.integers(0, 4, L).astype(np.uint8)
        r = float(rng.choice(rates))
        if r >= 1.0:
            P = rng.integers(0, 4, int(rng.integers(lmin, lmax + 1))).astype(np.uint8)
        else:
            bb = synth.from_lists([T], [T])
            P, _ = synth.mutate(rng, bb.txt, bb.txt_off, [r])
        pats.append(P)
        txts.append(T)
    return synth.from_lists(pats, txts)


@pytest.mark.parametrize("smax", [-1, 0, 1, 8, 41, 200, 201])  # odd ones: not multiples of gcd(4, 6, 2)
def test_thresholds_and_noise(ctx, smax):
    check(ctx, _mixed(41, 600, 0, 300, [0.0, 0.02, 0.08, 0.3, 1.0]), AFF, smax)


def test_degenerate_pairs(ctx):
    pats = ["", "", "A", "", "ACGT", "A" * 300, "", "ACGTACGT" * 40, "T" * 200, "G"]
    txts = ["", "A", "", "ACGTACGTAC", "", "", "C" * 257, "ACGTACGT" * 40, "A" * 200, "G" * 500]
    b = synth.from_lists(pats, txts)
    check(ctx, b)
    check(ctx, b, max_score=10)
    check(ctx, b, (0, 3, 4, 1))


def test_long_reads_vs_scalar_wfa(ctx):
    # 1-6 kbp at 1-10 %: the full store goes to HBM arenas; compared against
    # the scalar WFA, which the CPU suite pins to the Gotoh oracle
    b = _mixed(42, 24, 1000, 6000, [0.01, 0.05, 0.1])
    s, st, cg, off = run(ctx, b, "wfa", AFF)
    for i in range(b.n):
        ws, wsc, wr, _ = oracle.wfa_pair(b.pattern(i), b.text(i), AFF)
        assert (st[i], s[i]) == (ws, wsc), i
        assert cg[off[i]:off[i + 1]].tolist() == wr, i


def test_many_runs_spill_path(ctx):
    rng = np.random.default_rng(7)
    pats, txts = [], []
    for _ in range(64):
        T = rng.integers(0, 4, 160).astype(np.uint8)
        P = T.copy()
        P[::3] = (P[::3] + 1) % 4
        pats.append(P)
        txts.append(T)
    check(ctx, synth.from_lists(pats, txts), (0, 1, 6, 2))


def test_score_only_matches(ctx):
    b = synth.workload("wfa250", n=3000)
    full = run(ctx, b, "wfa", AFF, 200)
    s, st, _, off = run(ctx, b, "wfa", AFF, 200, want_cigar=False)
    assert np.array_equal(s, full[0]) and np.array_equal(st, full[1]) and not off.any()


def test_walk_fallback_to_full_store(ctx):
    # A small scratch limit leaves the HBM-ring pass too little room for the
    # origin codes of its longer pairs, which then take the full-store passes;
    # the shorter ones are walked from their codes.
    # (at 2 GiB each workgroup keeps under 3 MB of codes: the 10 % pairs of
    # 8-10 kbp need more, the 1 % pairs far less)
    b = _mixed(43, 12, 8000, 10000, [0.01, 0.1])
    small = aim.Context(0, scratch_limit=2 << 30)
    try:
        s, st, cg, off = run(small, b, "wfa", AFF)
    finally:
        small.close()
    for i in range(b.n):
        ws, wsc, wr, _ = oracle.wfa_pair(b.pattern(i), b.text(i), AFF)
        assert (st[i], s[i]) == (ws, wsc), i
        assert cg[off[i]:off[i + 1]].tolist() == wr, i


def test_one_wave_walk_score_cap():
    # Penalties with R = 32 and pairs of at most 127 bases stay in the
    # one-wavefront pass's window; scores of 2048 and more exceed the scores
    # whose origin codes it keeps, so those pairs take the full-store pass.
    pen = (0, 31, 20, 11)
    pats, txts = [], []
    rng = np.random.default_rng(12)
    for L in (100, 113, 120, 127):
        pats += [np.zeros(L, np.uint8), np.tile(np.array([0, 1], np.uint8), L // 2)]
        txts += [np.ones(L, np.uint8), np.tile(np.array([2, 3], np.uint8), L // 2)]
    for _ in range(24):
        pats.append(rng.integers(0, 4, int(rng.integers(60, 128))).astype(np.uint8))
        txts.append(rng.integers(0, 4, int(rng.integers(60, 128))).astype(np.uint8))
    b = synth.from_lists(pats, txts)
    want = oracle.align_batch(b, "wfa", pen)
    assert (want[0] >= 2048).sum() >= 4 and (want[0] < 2048).sum() >= 20
    c = aim.Context(0)
    try:
        check(c, b, pen)
    finally:
        c.close()


def test_reads_beyond_16bit_offsets(ctx):
    # A batch with reads over 32,000 bases takes the 32-bit paths throughout:
    # the LDS-ring score pass with the full-store walk for narrow pairs, and
    # the HBM-ring pass (32-bit ring, sequences read in place) with its code
    # walk for the rest; checked against the scalar WFA.
    rng = np.random.default_rng(44)
    pats, txts = [], []
    for L, r in [(33000, 0.001), (40000, 0.005), (36000, 0.003), (300, 0.02), (1200, 0.05), (50, 0.0)]:
        T = rng.integers(0, 4, L).astype(np.uint8)
        bb = synth.from_lists([T], [T])
        P, _ = synth.mutate(rng, bb.txt, bb.txt_off, [r])
        pats.append(P)
        txts.append(T)
    b = synth.from_lists(pats, txts)
    s, st, cg, off = run(ctx, b, "wfa", AFF)
    for i in range(b.n):
        ws, wsc, wr, _ = oracle.wfa_pair(b.pattern(i), b.text(i), AFF)
        assert (st[i], s[i]) == (ws, wsc), i
        assert cg[off[i]:off[i + 1]].tolist() == wr, i


@pytest.mark.parametrize("smax", [-1, 600])
@pytest.mark.parametrize("pen", [(0, 41, 10, 29), (0, 40, 10, 30)])
def test_large_ring_penalties(ctx, smax, pen):
    # (0, 41, 10, 29): max(x, o + e) = 41, a ring of 42 scores, beyond the
    # one-wavefront pass, so the LDS-ring and HBM-ring score passes and the
    # full-store walk run.  (0, 40, 10, 30) has the common divisor 10 and runs
    # as (4, 1, 3) in the one-wavefront pass.
    check(ctx, _mixed(45, 300, 0, 400, [0.0, 0.02, 0.1, 1.0]), pen, smax)


def _long_run_pairs(seed):
    """Pairs whose alignments hold match runs longer than 1,024 bases (the
    replay extends a run one wavefront round per 1,024 bases): identical pairs
    around multiples of 16 and 1,024 bases, one mismatch on either side of those
    boundaries, and dense-edit blocks (10 %) between identical runs of
    1,024-2,100 bases, wide enough to leave the one-wavefront window."""
    rng = np.random.default_rng(seed)

    def rand(n):
        return "".join(rng.choice(list("ACGT"), n))

    def dense(s, rate):
        out = []
        for c in s:
            r = rng.random()
            if r < rate / 3:
                out.append("ACGT"[("ACGT".index(c) + 1 + int(rng.integers(3))) % 4])
            elif r < 2 * rate / 3:
                out.append(c + "ACGT"[int(rng.integers(4))])
            elif r >= rate:
                out.append(c)
        return "".join(out)

    pats, txts = [], []
    for L in (1023, 1024, 1025, 1040, 2048, 3001):
        t = rand(L)
        pats.append(t)
        txts.append(t)
    for pos in (16, 1023, 1024, 1025, 2047, 3999):
        t = rand(4000)
        p = t[:pos] + "ACGT"[("ACGT".index(t[pos]) + 1) % 4] + t[pos + 1:]
        pats.append(p)
        txts.append(t)
    for run_len in (1024, 1025, 1500, 2100):
        blocks_t, blocks_p = [], []
        for _ in range(3):
            a = rand(700)
            blocks_t.append(a)
            blocks_p.append(dense(a, 0.10))
            r = rand(run_len)
            blocks_t.append(r)
            blocks_p.append(r)
        pats.append("".join(blocks_p))
        txts.append("".join(blocks_t))
    return synth.from_lists(pats, txts)


def test_long_match_runs(ctx):
    b = _long_run_pairs(2024)
    s, st, cg, off = run(ctx, b, "wfa", AFF)
    stats = ctx.last_call_stats()
    # the dense-block pairs leave the one-wavefront window: their walks run in
    # the window classes, the others' in the one-wavefront pass
    assert sum(stats["wfa_class_pairs"]) >= 1, stats
    assert stats["wfa_walk_failed"] == 0, stats
    for i in range(b.n):
        ws, wsc, wr, _ = oracle.wfa_pair(b.pattern(i), b.text(i), AFF)
        assert (st[i], s[i]) == (ws, wsc), i
        assert cg[off[i]:off[i + 1]].tolist() == wr, i
    # the same pairs through WFA-adaptive (the class kernel's walk with the
    # reduction step) against the adaptive oracle
    ctx.wfa_adaptive_params(10, 50)
    got = run(ctx, b, "wfa_adaptive", AFF)
    want = oracle.wfa_batch(b, AFF, -1, adaptive=(10, 50))
    bad = compare(got, want)
    assert not bad, "%d mismatches, first: %s" % (len(bad), describe(b, bad[0], got, want))
