"""The memory-bounded pass for long WFA pairs (k_wfa_long): pairs whose
origin codes and full store fit no slot get their CIGAR from checkpoints of
the wavefront ring and windows of recomputed codes; the same pass re-runs, in
place, pairs whose runs outgrow their slot and the run pool.  Scores,
statuses and CIGARs against the scalar wavefront oracle, element by element.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
import synth  # noqa: E402
import paper_2208_01243_amd as aim  # noqa: E402
from gpu_util import compare, describe, run  # noqa: E402

AFF = (0, 4, 6, 2)


def _pairs(seed, lens_rates):
    rng = np.random.default_rng(seed)
    pats, txts = [], []
    for L, r in lens_rates:
        T = rng.integers(0, 4, L).astype(np.uint8)
        bb = synth.from_lists([T], [T])
        P, _ = synth.mutate(rng, bb.txt, bb.txt_off, [r])
        pats.append(P)
        txts.append(T)
    return synth.from_lists(pats, txts)


def check(c, b, pen=AFF, max_score=-1):
    print("batch of %d pairs, max_len %d" % (b.n, max(b.pat_len.max(), b.txt_len.max())), flush=True)
    got = run(c, b, "wfa", pen, max_score)
    want = oracle.wfa_batch(b, pen, max_score)
    bad = compare(got, want)
    assert not bad, "%d mismatches, first: %s" % (len(bad), describe(b, bad[0], got, want))
    return got


def test_long_pairs_past_every_store_class():
    # 10 kbp at 20 %: full stores of ~65 M words, past the largest class of a
    # context hard-limited to 1 GiB (~34 M words), so these pairs are walked
    # by the long pass; short pairs in the same batch take the usual passes
    rng = np.random.default_rng(41)
    spec = [(10000, 0.20)] * 4 + [(int(rng.integers(100, 2000)), float(rng.uniform(0, 0.1))) for _ in range(40)]
    b = _pairs(41, spec)
    with aim.Context(0, scratch_limit=1 << 30, hard_limit=True) as c:
        got = check(c, b)
        st = c.last_call_stats()
        assert st["wfa_long_pairs"] >= 1, st
        assert st["wfa_long_failed"] == 0, st
        assert (got[1] == 0).all()


def test_long_pairs_with_threshold_and_other_penalties():
    spec = [(9000, 0.18)] * 3 + [(300, 0.05)] * 10
    b = _pairs(42, spec)
    with aim.Context(0, scratch_limit=1 << 30, hard_limit=True) as c:
        for pen, smax in [(AFF, 20000), ((0, 3, 4, 1), -1)]:
            check(c, b, pen, smax)
            assert c.last_call_stats()["wfa_long_failed"] == 0


def test_runs_beyond_slot_and_pool_are_rerun():
    # 600 pairs of 4-5 kbp at 15-30 % error reserve thousands of pool words
    # each: a 256 MiB scratch limit leaves a pool of 2^20 words, which they
    # exhaust, so some are re-aligned in place (by the long pass)
    rng = np.random.default_rng(43)
    spec = [(int(rng.integers(4000, 5001)), float(rng.uniform(0.15, 0.3))) for _ in range(600)]
    b = _pairs(43, spec)
    with aim.Context(0, scratch_limit=256 << 20) as c:
        check(c, b)
        st = c.last_call_stats()
        assert st["cigar_reruns"] > 0, st
        assert st["wfa_long_failed"] == 0, st
