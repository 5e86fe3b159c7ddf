"""Full-size workloads in the launch configuration bench.py times.

Every pair is checked against properties that hold at any size (each CIGAR
consumes exactly its pair's bases, its rescored cost equals the reported
score, statuses are consistent); a seeded random sample of pairs is compared
bit for bit with the oracle, pair by pair.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
import synth  # noqa: E402
import paper_2208_01243_amd as aim  # noqa: E402
from gpu_util import run  # noqa: E402


def vector_invariants(batch, score, status, cigar, off, pen):
    """CIGAR consumption and gap-model cost for every aligned pair, vectorised."""
    _, x, o, e = pen
    ok = status == aim.PAIR_ALIGNED
    nr = np.diff(off)
    assert (nr[~ok] == 0).all()
    runs = cigar[:off[-1]].astype(np.int64)
    op, ln = runs & 15, runs >> 4
    assert (op <= 3).all() and (ln > 0).all()
    pair = np.repeat(np.arange(batch.n), nr)
    cons_p = np.bincount(pair, weights=ln * ((op == 0) | (op == 1) | (op == 2)), minlength=batch.n)
    cons_t = np.bincount(pair, weights=ln * ((op == 0) | (op == 1) | (op == 3)), minlength=batch.n)
    cost = np.bincount(pair, weights=np.where(op == 1, x * ln, np.where(op >= 2, o + e * ln, 0)),
                       minlength=batch.n)
    assert np.array_equal(cons_p[ok], batch.pat_len[ok]) and np.array_equal(cons_t[ok], batch.txt_len[ok])
    assert np.array_equal(cost[ok].astype(np.int64), score[ok].astype(np.int64))
    # adjacent runs never repeat an op
    same = (op[1:] == op[:-1]) & (pair[1:] == pair[:-1])
    assert not same.any()


@pytest.mark.parametrize("name,sample", [("swg150", 3000), ("wfa250", 3000), ("nw100", 10_000)])
def test_full_workload(name, sample):
    w = synth.WORKLOADS[name]
    b = synth.workload(name)
    print("full workload %s: %d pairs" % (name, b.n), flush=True)
    with aim.Context(0) as ctx:
        s, st, cg, off = run(ctx, b, w["alg"], w["pen"], w["max_score"], enc=w["enc"])
        stats = ctx.last_call_stats()
    # a fused walk over kept origin codes never fails
    assert stats["wfa_walk_failed"] == 0, stats
    assert (st != aim.PAIR_INVALID).all() and (st != aim.PAIR_CIGAR_OVERFLOW).all()
    vector_invariants(b, s, st, cg, off, w["pen"])
    rng = np.random.default_rng(99)
    idx = np.sort(rng.choice(b.n, size=min(sample, b.n), replace=False))
    sub = b.subset(idx)
    ws, wst, wc, wo = oracle.align_batch(sub, w["alg"], w["pen"], w["max_score"])
    for t, i in enumerate(idx):
        assert (s[i], st[i]) == (ws[t], wst[t]), (name, i)
        assert np.array_equal(cg[off[i]:off[i + 1]], wc[wo[t]:wo[t + 1]]), (name, i)


def test_repeat_calls_swg150():
    # The warm path: scratch no longer grows, so nothing synchronises inside a
    # call and the first tier's traceback (second stream) runs beside the
    # escalation tiers.  Both calls must give the same, valid results.
    w = synth.WORKLOADS["swg150"]
    b = synth.workload("swg150")
    with aim.Context(0) as ctx:
        first = run(ctx, b, w["alg"], w["pen"], w["max_score"], enc=w["enc"])
        second = run(ctx, b, w["alg"], w["pen"], w["max_score"], enc=w["enc"])
    for s, st, cg, off in (first, second):
        vector_invariants(b, s, st, cg, off, w["pen"])
    assert all(np.array_equal(u, v) for u, v in zip(first, second))


def test_full_wfa_mixed():
    # The batching-form workload in the call bench.py times: all 500,000 pairs
    # (100 bp - 10 kbp, 0.5 - 10 %) in one call.  Every pair is checked by the
    # vectorised invariants; a seeded sample spread over the whole index range
    # is compared bit for bit: pairs up to 2,500 bp with the full-matrix
    # oracle, longer ones with the scalar wavefront oracle.
    from concurrent.futures import ThreadPoolExecutor
    w = synth.WORKLOADS["wfa_mixed"]
    b = synth.workload("wfa_mixed")
    print("full workload wfa_mixed: %d pairs" % b.n, flush=True)
    with aim.Context(0) as ctx:
        s, st, cg, off = run(ctx, b, "wfa", w["pen"], w["max_score"])
        stats = ctx.last_call_stats()
    print("path counters", stats, flush=True)
    assert stats["wfa_walk_failed"] == 0, stats
    assert (st == aim.PAIR_ALIGNED).all()
    vector_invariants(b, s, st, cg, off, w["pen"])
    rng = np.random.default_rng(2024)
    L = np.maximum(b.pat_len, b.txt_len)
    short = np.nonzero(L <= 2500)[0]
    longi = np.nonzero(L > 2500)[0]
    idx_s = np.sort(rng.choice(short, size=400, replace=False))
    idx_l = np.sort(rng.choice(longi, size=60, replace=False))
    sub = b.subset(idx_s)
    ws, wst, wc, wo = oracle.align_batch(sub, "wfa", w["pen"], -1)
    for t, i in enumerate(idx_s):
        assert (s[i], st[i]) == (ws[t], wst[t]), i
        assert np.array_equal(cg[off[i]:off[i + 1]], wc[wo[t]:wo[t + 1]]), i

    def one(i):
        return oracle.wfa_pair(b.pattern(i), b.text(i), w["pen"])

    with ThreadPoolExecutor(8) as ex:
        res = list(ex.map(one, idx_l))
    for i, r in zip(idx_l, res):
        assert (st[i], s[i]) == (r[0], r[1]) and cg[off[i]:off[i + 1]].tolist() == r[2], i


@pytest.mark.parametrize("name,sample", [("wfa_adaptive_150", 3000), ("wfa_adaptive_1k", 600),
                                         ("wfa_adaptive_10k", 60), ("genasm150", 3000), ("genasm1k", 600)])
def test_full_heuristic_workload(name, sample):
    # WFA-adaptive and GenASM at full size, in the call bench.py times: every
    # pair by the vectorised invariants (a heuristic's alignment is still a
    # valid alignment whose cost is its score), a seeded sample bit for bit
    # against the algorithm's own oracle
    w = synth.WORKLOADS[name]
    b = synth.workload(name)
    print("full workload %s: %d pairs" % (name, b.n), flush=True)
    with aim.Context(0) as ctx:
        if w["alg"] == "wfa_adaptive":
            ctx.wfa_adaptive_params(*w["adaptive"])
        s, st, cg, off = run(ctx, b, w["alg"], w["pen"], w["max_score"], enc=w["enc"])
        stats = ctx.last_call_stats()
    assert stats["wfa_walk_failed"] == 0, stats
    assert (st != aim.PAIR_INVALID).all() and (st != aim.PAIR_CIGAR_OVERFLOW).all()
    if w["alg"] == "wfa_adaptive":
        assert (st == aim.PAIR_ALIGNED).all() and stats["wfa_adaptive_dropped"] > 0, stats
    vector_invariants(b, s, st, cg, off, w["pen"])
    rng = np.random.default_rng(7)
    idx = np.sort(rng.choice(b.n, size=min(sample, b.n), replace=False))
    sub = b.subset(idx)
    if w["alg"] == "genasm":
        ws, wst, wc, wo = oracle.genasm_batch(sub, w["max_score"])
    else:
        ws, wst, wc, wo = oracle.wfa_batch(sub, w["pen"], w["max_score"], adaptive=w["adaptive"])
    for t, i in enumerate(idx):
        assert (s[i], st[i]) == (ws[t], wst[t]), (name, i)
        assert np.array_equal(cg[off[i]:off[i + 1]], wc[wo[t]:wo[t + 1]]), (name, i)
