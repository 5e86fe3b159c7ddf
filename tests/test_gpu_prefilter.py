"""The exact pre-alignment filter on the GPU (aim_prefilter, and the filter
in front of aim_align_batch) against the CPU oracle.

aim_prefilter's lower bounds must equal oracle.prefilter.lower_bounds
element by element; every pair it rejects must have an oracle optimum above
the threshold; and aim_align_batch must return the same results, bit for
bit, with and without the filter.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
import synth  # noqa: E402
import paper_2208_01243_amd as aim  # noqa: E402
from gpu_util import compare, describe, run, to_device  # noqa: E402
from oracle.prefilter import REACH, lower_bounds  # noqa: E402

PENS = [("wfa", (0, 4, 6, 2)), ("swg", (0, 3, 4, 1)), ("nw", (0, 1, 0, 1)), ("nw", (0, 3, 0, 4)),
        ("swg", (0, 9, 1, 1)), ("swg", (0, 1, 5, 3))]


@pytest.fixture(scope="module")
def ctx():
    c = aim.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def ctx_nofilter():
    c = aim.Context(0, prefilter=False)
    yield c
    c.close()


def gpu_lower(ctx, batch, alg, pen, max_score, enc="2bit", max_len=None):
    dev, e = to_device(batch, enc)
    if max_len is None:
        max_len = int(max(batch.pat_len.max(initial=0), batch.txt_len.max(initial=0)))
    n = batch.n
    lower = torch.full((max(n, 1),), -7, dtype=torch.int32, device="cuda")
    passed = torch.full((max(n, 1),), 7, dtype=torch.int8, device="cuda")
    ctx.prefilter(*dev, enc=e, max_len=max_len, alg=alg, pen=pen, max_score=max_score, lower=lower,
                  passed=passed)
    torch.cuda.synchronize()
    return lower.cpu().numpy()[:n], passed.cpu().numpy()[:n]


def mixed_batch(seed, n, lmax, unrelated=0.3):
    rng = np.random.default_rng(seed)
    pats, txts = [], []
    for _ in range(n):
        L = int(rng.integers(0, lmax + 1))
        T = rng.integers(0, 4, L).astype(np.uint8)
        u = rng.random()
        if u < unrelated:
            P = rng.integers(0, 4, int(rng.integers(0, lmax + 1))).astype(np.uint8)
        else:
            bb = synth.from_lists([T], [T])
            P, _ = synth.mutate(rng, bb.txt, bb.txt_off, [float(rng.uniform(0, 0.2))])
        pats.append(P)
        txts.append(T)
    return synth.from_lists(pats, txts)


@pytest.mark.parametrize("alg,pen", PENS)
def test_lower_bounds_match_oracle(ctx, alg, pen):
    # short reads: the 8-word kernel; several waves, ragged tail
    b = mixed_batch(1, 3001, 250)
    lo, ps = gpu_lower(ctx, b, alg, pen, 150)
    want = lower_bounds(b, alg, pen)
    assert np.array_equal(lo, want), np.nonzero(lo != want)[0][:10]
    assert np.array_equal(ps, (want <= 150).astype(np.int8))


def test_lower_bounds_long_and_reach(ctx):
    # up to 1,100 bases: the 32-word kernel, the reach boundary on both sides
    rng = np.random.default_rng(2)
    b0 = mixed_batch(3, 600, 1100)
    extra_p, extra_t = [], []
    for sl, tl in [(REACH, REACH), (REACH, REACH + 40), (REACH + 1, REACH + 1), (REACH + 1, REACH + 9),
                   (REACH - 1, REACH + 60), (993, 1024), (1, 1100), (0, 1100), (1100, 0), (32, 1), (33, 64)]:
        t = rng.integers(0, 4, tl).astype(np.uint8)
        p = rng.integers(0, 4, sl).astype(np.uint8)
        extra_p += [p, t]
        extra_t += [t, p]
    pats = [b0.pattern(i) for i in range(b0.n)] + extra_p
    txts = [b0.text(i) for i in range(b0.n)] + extra_t
    b = synth.from_lists(pats, txts)
    for alg, pen in [("wfa", (0, 4, 6, 2)), ("nw", (0, 1, 0, 1))]:
        lo, ps = gpu_lower(ctx, b, alg, pen, -1)
        want = lower_bounds(b, alg, pen)
        assert np.array_equal(lo, want), np.nonzero(lo != want)[0][:10]
        assert (ps == 1).all()


@pytest.mark.parametrize("enc", ["ascii", "code"])
def test_encodings_and_invalid(ctx, enc):
    b = mixed_batch(4, 700, 200)
    lo, ps = gpu_lower(ctx, b, "swg", (0, 4, 6, 2), 60, enc=enc)
    want = lower_bounds(b, "swg", (0, 4, 6, 2))
    assert np.array_equal(lo, want)
    assert np.array_equal(ps, (want <= 60).astype(np.int8))
    # a pair beyond max_len is invalid: lower -1, pass 0
    lo2, ps2 = gpu_lower(ctx, b, "swg", (0, 4, 6, 2), 60, enc=enc, max_len=150)
    bad = (b.pat_len > 150) | (b.txt_len > 150)
    assert bad.any() and (lo2[bad] == -1).all() and (ps2[bad] == 0).all()
    assert np.array_equal(lo2[~bad], want[~bad])


def test_non_acgt_is_invalid(ctx):
    b = synth.from_lists(["ACGT", "ACGT", "AC"], ["ACGA", "ACGT", "ACGT"])
    dev, e = to_device(b, "ascii")
    dev[0][1] = ord("N")  # second base of the first pattern
    lower = torch.empty(3, dtype=torch.int32, device="cuda")
    passed = torch.empty(3, dtype=torch.int8, device="cuda")
    ctx.prefilter(*dev, enc=e, max_len=4, alg="swg", pen=(0, 4, 6, 2), max_score=-1, lower=lower, passed=passed)
    torch.cuda.synchronize()
    assert lower.cpu().tolist() == [-1, 0, 6 + 2 * 2] and passed.cpu().tolist() == [0, 1, 1]


def test_empty_batch(ctx):
    b = synth.from_lists([], [])
    lo, ps = gpu_lower(ctx, b, "nw", (0, 1, 0, 1), 3)
    assert len(lo) == 0 and len(ps) == 0


def test_rejections_are_sound(ctx):
    # every pair the filter drops has an optimum above the threshold
    b = mixed_batch(5, 2000, 300, unrelated=0.5)
    for alg, pen, S in [("wfa", (0, 4, 6, 2), 200), ("swg", (0, 1, 5, 3), 90), ("nw", (0, 3, 0, 4), 100)]:
        lo, ps = gpu_lower(ctx, b, alg, pen, S)
        opt = oracle.align_batch(b, "nw" if alg == "nw" else "swg", pen, -1, want_cigar=False)[0]
        assert (lo <= opt).all()
        assert (opt[ps == 0] > S).all()
        assert (ps == 0).sum() > 0


@pytest.mark.parametrize("alg,pen,S", [("wfa", (0, 4, 6, 2), 200), ("swg", (0, 4, 6, 2), 60),
                                       ("nw", (0, 1, 0, 1), 5), ("wfa", (0, 1, 5, 3), 40)])
def test_align_batch_same_with_and_without_filter(ctx, ctx_nofilter, alg, pen, S):
    b = mixed_batch(6, 2500, 400, unrelated=0.3)
    got = run(ctx, b, alg, pen, S)
    plain = run(ctx_nofilter, b, alg, pen, S)
    want = oracle.align_batch(b, alg, pen, S)
    bad = compare(got, want)
    assert not bad, describe(b, bad[0], got, want)
    assert not compare(plain, want)
    st = ctx.last_call_stats()
    lo = lower_bounds(b, alg, pen)
    valid = np.ones(b.n, bool)
    assert st["prefilter_rejected"] == int(((lo > S) & valid).sum())


def test_wfa250_slice(ctx):
    w = synth.WORKLOADS["wfa250"]
    b = synth.workload("wfa250", n=20_000)
    got = run(ctx, b, "wfa", w["pen"], w["max_score"])
    want = oracle.align_batch(b, "wfa", w["pen"], w["max_score"])
    bad = compare(got, want)
    assert not bad, describe(b, bad[0], got, want)
    st = ctx.last_call_stats()
    # the unrelated fifth is rejected up front
    assert st["prefilter_rejected"] >= 0.19 * b.n
