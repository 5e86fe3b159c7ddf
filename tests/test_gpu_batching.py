"""Batching form: length-sorted queues, autotuned launch parameters and
captured HIP graphs, each bit-exact against the oracle."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
import synth  # noqa: E402
import paper_2208_01243_amd as aim  # noqa: E402
from gpu_util import compare, describe, run, to_device  # noqa: E402


def _outputs(b):
    n = b.n
    score = torch.empty(n, dtype=torch.int32, device="cuda")
    status = torch.empty(n, dtype=torch.int8, device="cuda")
    cap = int((b.pat_len.astype(np.int64) + b.txt_len + 1).sum()) + 1
    cigar = torch.empty(cap, dtype=torch.int32, device="cuda")
    off = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    return score, status, cigar, off


def _host(outs):
    s, st, cg, off = outs
    torch.cuda.synchronize()
    return s.cpu().numpy(), st.cpu().numpy(), cg.cpu().numpy().view(np.uint32), off.cpu().numpy()


def _same_shape_batch(b, seed):
    """A batch with the same lengths as b but different bases."""
    rng = np.random.default_rng(seed)
    pat = b.pat.copy()
    txt = b.txt.copy()
    flip = rng.random(len(txt)) < 0.03
    txt[flip] = (txt[flip] + 1) % 4
    flip = rng.random(len(pat)) < 0.03
    pat[flip] = (pat[flip] + 2) % 4
    return synth.PairBatch(pat, b.pat_off.copy(), txt, b.txt_off.copy())


@pytest.mark.parametrize("name", ["nw100", "swg150"])
def test_graph_replays(name):
    w = synth.WORKLOADS[name]
    b = synth.workload(name, n=4000)
    dev, enc = to_device(b, w["enc"])
    outs = _outputs(b)
    max_len = int(max(b.pat_len.max(), b.txt_len.max()))
    stream = torch.cuda.Stream()
    with aim.Context(0) as ctx, torch.cuda.stream(stream):
        g = ctx.graph_capture(*dev, enc=enc, max_len=max_len, alg=w["alg"], pen=w["pen"],
                              max_score=w["max_score"], score=outs[0], status=outs[1], cigar=outs[2],
                              cigar_off=outs[3], stream=stream)
        want = oracle.align_batch(b, w["alg"], w["pen"], w["max_score"])
        for rep in range(3):
            for t in outs:
                t.zero_()  # eager work between replays
            stream.synchronize()
            g.launch(stream)
            got = _host(outs)
            bad = compare(got, want)
            assert not bad, (rep, describe(b, bad[0], got, want))
        # new contents in the captured input buffers: the replay aligns them
        b2 = _same_shape_batch(b, 3)
        dev2, _ = to_device(b2, w["enc"])
        for dst, src in zip(dev, dev2):
            dst.copy_(src)
        stream.synchronize()
        g.launch(stream)
        got = _host(outs)
        want2 = oracle.align_batch(b2, w["alg"], w["pen"], w["max_score"])
        bad = compare(got, want2)
        assert not bad, describe(b2, bad[0], got, want2)
        g.close()


@pytest.mark.parametrize("name,n", [("swg150", 20000), ("wfa250", 5000)])
def test_autotune_is_exact_and_cached(name, n, tmp_path):
    w = synth.WORKLOADS[name]
    b = synth.workload(name, n=n)
    dev, enc = to_device(b, w["enc"])
    outs = _outputs(b)
    max_len = int(max(b.pat_len.max(), b.txt_len.max()))
    with aim.Context(0) as ctx:
        params, ms = ctx.autotune(*dev, enc=enc, max_len=max_len, alg=w["alg"], pen=w["pen"],
                                  max_score=w["max_score"], score=outs[0], status=outs[1],
                                  cigar=outs[2], cigar_off=outs[3], reps=1)
        assert ms > 0 and ctx.tune_get(w["alg"], max_len) == params
        want = oracle.align_batch(b, w["alg"], w["pen"], w["max_score"])
        bad = compare(_host(outs), want)
        assert not bad
        path = str(tmp_path / "tune.txt")
        ctx.tune_save(path)
    with aim.Context(0) as ctx2:
        ctx2.tune_load(path)
        assert ctx2.tune_get(w["alg"], max_len) == params
        got = run(ctx2, b, w["alg"], w["pen"], w["max_score"], enc=w["enc"])
        assert not compare(got, want)


def _mixed(seed, count, lmin, lmax, rates):
    rng = np.random.default_rng(seed)
    pats, txts = [], []
    for _ in range(count):
        L = int(np.exp(rng.uniform(np.log(lmin), np.log(lmax))))
        T = rng.integers(0, 4, L).astype(np.uint8)
        bb = synth.from_lists([T], [T])
        P, _ = synth.mutate(rng, bb.txt, bb.txt_off, [float(rng.choice(rates))])
        pats.append(P)
        txts.append(T)
    return synth.from_lists(pats, txts)


@pytest.mark.parametrize("alg,pen", [("swg", (0, 4, 6, 2)), ("nw", (0, 1, 0, 1)), ("wfa", (0, 4, 6, 2))])
@pytest.mark.parametrize("sort", [0, 1])
def test_length_sort_exact(alg, pen, sort):
    b = _mixed(50, 1500, 20, 1200, [0.005, 0.02, 0.06])
    with aim.Context(0) as ctx:
        L = int(max(b.pat_len.max(), b.txt_len.max()))
        p = ctx.tune_get(alg, L)
        p[2] = sort
        ctx.tune_set(alg, L, p)
        got = run(ctx, b, alg, pen)
    want = oracle.align_batch(b, alg, pen)
    bad = compare(got, want)
    assert not bad, describe(b, bad[0], got, want)


@pytest.mark.parametrize("alg,pen", [("swg", (0, 4, 6, 2)), ("nw", (0, 1, 0, 1))])
@pytest.mark.parametrize("band16", [0, 1, 2, 3])
def test_first_tier_variants_exact(alg, pen, band16):
    # the first band tier in 32-bit cells (0), packed 16-bit cells walked by the
    # fill itself (1), by a separate kernel beside the escalation tiers (2), or
    # the size-dependent default (3, the fill's own walk at this batch size);
    # two calls in one context so the second runs on warm scratch
    b = _mixed(51, 4000, 60, 260, [0.0, 0.02, 0.05, 0.12])
    with aim.Context(0) as ctx:
        L = int(max(b.pat_len.max(), b.txt_len.max()))
        p = ctx.tune_get(alg, L)
        p[6] = band16
        ctx.tune_set(alg, L, p)
        run(ctx, b, alg, pen)
        got = run(ctx, b, alg, pen)
    want = oracle.align_batch(b, alg, pen)
    bad = compare(got, want)
    assert not bad, describe(b, bad[0], got, want)


def test_wfa_mixed_sample():
    # the batching-form workload (100 bp - 10 kbp, 0.5-10 %): first 3000 pairs,
    # checked pair by pair (pairs above 2.5 kbp against the scalar WFA)
    w = synth.WORKLOADS["wfa_mixed"]
    b = synth.workload("wfa_mixed", n=3000)
    with aim.Context(0) as ctx:
        s, st, cg, off = run(ctx, b, "wfa", w["pen"], w["max_score"])
    short = np.nonzero(np.maximum(b.pat_len, b.txt_len) <= 2500)[0]
    sub = b.subset(short)
    ws, wst, wc, wo = oracle.align_batch(sub, "wfa", w["pen"], -1)
    for t, i in enumerate(short):
        assert (s[i], st[i]) == (ws[t], wst[t]) and np.array_equal(cg[off[i]:off[i + 1]], wc[wo[t]:wo[t + 1]]), i
    longi = np.nonzero(np.maximum(b.pat_len, b.txt_len) > 2500)[0]
    rng = np.random.default_rng(1)
    for i in rng.choice(longi, size=min(40, len(longi)), replace=False):
        r = oracle.wfa_pair(b.pattern(i), b.text(i), w["pen"])
        assert (st[i], s[i]) == (r[0], r[1]) and cg[off[i]:off[i + 1]].tolist() == r[2], i


def _capture(ctx, b, w, stream):
    dev, enc = to_device(b, w["enc"])
    outs = _outputs(b)
    max_len = int(max(b.pat_len.max(), b.txt_len.max()))
    g = ctx.graph_capture(*dev, enc=enc, max_len=max_len, alg=w["alg"], pen=w["pen"],
                          max_score=w["max_score"], score=outs[0], status=outs[1], cigar=outs[2],
                          cigar_off=outs[3], stream=stream)
    return g, dev, outs, max_len, enc


@pytest.mark.parametrize("name,n", [("swg150", 70_000), ("wfa250", 20_000), ("wfa_mixed", 3000)])
def test_graph_replays_large_and_wfa(name, n):
    # swg150 at 70,000 pairs takes the two-stream path (the first tier's walk
    # on the context's second stream beside the escalation tiers), which the
    # capture must record as graph dependencies; the WFA batches capture the
    # wavefront passes and their fallbacks.  Every replay, with eager work
    # between them, must reproduce the eager call.
    w = dict(synth.WORKLOADS[name])
    b = synth.workload(name, n=n)
    print("graph replays: %s, %d pairs" % (name, n), flush=True)
    stream = torch.cuda.Stream()
    with aim.Context(0) as ctx, torch.cuda.stream(stream):
        g, dev, outs, max_len, enc = _capture(ctx, b, w, stream)
        want = _host(outs)
        idx = np.arange(0, n, max(1, n // 300))
        sub = b.subset(idx)
        ws, wst, wc, wo = oracle.align_batch(sub, w["alg"], w["pen"], w["max_score"])
        s, st, cg, off = want
        for t, i in enumerate(idx):
            assert (s[i], st[i]) == (ws[t], wst[t]) and np.array_equal(cg[off[i]:off[i + 1]], wc[wo[t]:wo[t + 1]])
        for rep in range(3):
            for t in outs:
                t.zero_()
            stream.synchronize()
            g.launch(stream)
            got = _host(outs)
            assert all(np.array_equal(u, v) for u, v in zip(got, want)), rep
        g.close()


def test_graph_replay_on_another_stream_between_eager_calls():
    # a replay shares the context's scratch with its eager calls: replays on a
    # second stream interleaved with eager calls on the first (no host sync
    # between them) must each give the eager results
    w = synth.WORKLOADS["swg150"]
    b = synth.workload("swg150", n=70_000)
    b2 = synth.workload("swg150", start=70_000, n=90_000)  # larger: the eager call grows scratch
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    with aim.Context(0) as ctx:
        with torch.cuda.stream(s1):
            g, dev, outs, max_len, enc = _capture(ctx, b, w, s1)
        want = _host(outs)
        want2 = oracle.align_batch(b2.subset(np.arange(0, b2.n, 300)), w["alg"], w["pen"], w["max_score"])
        outs2 = _outputs(b2)
        dev2, _ = to_device(b2, w["enc"])
        max_len2 = int(max(b2.pat_len.max(), b2.txt_len.max()))
        for rep in range(2):
            for t in outs:
                t.zero_()
            torch.cuda.synchronize()
            g.launch(s2)  # replay on s2
            # eager call on s1 right behind it (same context): must wait for the replay
            ctx.align_batch(*dev2, enc=enc, max_len=max_len2, alg=w["alg"], pen=w["pen"], max_score=w["max_score"],
                            score=outs2[0], status=outs2[1], cigar=outs2[2], cigar_off=outs2[3], stream=s1)
            torch.cuda.synchronize()
            got = _host(outs)
            assert all(np.array_equal(u, v) for u, v in zip(got, want)), rep
            g2 = _host(outs2)
            idx = np.arange(0, b2.n, 300)
            s, st, cg, off = g2
            ws, wst, wc, wo = want2
            for t, i in enumerate(idx):
                assert (s[i], st[i]) == (ws[t], wst[t]) and np.array_equal(cg[off[i]:off[i + 1]], wc[wo[t]:wo[t + 1]])
            if rep == 0:
                # the eager call grew the scratch: the graph is refused until captured again
                with pytest.raises(aim.AimError):
                    g.launch(s2)
                g.close()
                with torch.cuda.stream(s1):
                    g, dev, outs, max_len, enc = _capture(ctx, b, w, s1)
        g.close()


def test_hard_scratch_limit():
    # AIM_FLAG_HARD_LIMIT: the context's scratch never passes the limit; a
    # batch that would need more fails with AIM_ERR_OOM, and the context then
    # still aligns a batch that fits, with the same results as an unbounded one
    limit = 1 << 30
    b = synth.workload("wfa_mixed", n=3000)
    w = synth.WORKLOADS["wfa_mixed"]
    with aim.Context(0, scratch_limit=limit, hard_limit=True) as hc, aim.Context(0) as free:
        got = run(hc, b, "wfa", w["pen"], -1)
        assert not compare(got, run(free, b, "wfa", w["pen"], -1))
        cur, peak = hc.scratch_usage()
        assert 0 < cur <= peak <= limit
        assert free.scratch_usage()[1] > 0
    # 64 MiB: 200,000 pairs need more (their run slots alone take 100 MB)
    with aim.Context(0, scratch_limit=64 << 20, hard_limit=True) as hc:
        big = synth.workload("swg150", n=200_000)
        with pytest.raises(aim.AimError) as ei:
            run(hc, big, "swg", (0, 4, 6, 2), -1)
        assert ei.value.code == -3
        assert hc.scratch_usage()[1] <= 64 << 20
        small = synth.workload("swg150", n=5000)
        assert not compare(run(hc, small, "swg", (0, 4, 6, 2), -1), oracle.align_batch(small, "swg", (0, 4, 6, 2), -1))
        assert hc.scratch_usage()[1] <= 64 << 20


def test_autotune_wfa_mixed_per_bucket(tmp_path):
    # one mixed batch (100 bp - 10 kbp): the tuner keeps a batch tune and a
    # tune per window-class length bucket; the tuned calls return exactly what
    # the untuned ones do (a sample of which the scalar WFA oracle checks)
    w = synth.WORKLOADS["wfa_mixed"]
    b = synth.workload("wfa_mixed", n=20000)
    dev, enc = to_device(b, w["enc"])
    L = int(max(b.pat_len.max(), b.txt_len.max()))
    with aim.Context(0) as ref:
        want = run(ref, b, "wfa", w["pen"], -1, dev=(dev, enc))
    outs = _outputs(b)
    with aim.Context(0) as ctx:
        params, ms = ctx.autotune(*dev, enc=enc, max_len=L, alg="wfa", pen=w["pen"], max_score=-1,
                                  score=outs[0], status=outs[1], cigar=outs[2], cigar_off=outs[3], reps=1)
        assert ms > 0 and ctx.tune_get("wfa", L) == params
        assert not compare(_host(outs), want)
        ents = ctx.tune_entries()
        assert len([e for e in ents if e[0] == 1 and e[1] == aim.WFA_AFFINE]) >= 2, ents
        assert not compare(run(ctx, b, "wfa", w["pen"], -1, dev=(dev, enc)), want)
        path = str(tmp_path / "tune.txt")
        ctx.tune_save(path)
    with aim.Context(0) as ctx2:
        ctx2.tune_load(path)
        assert sorted(ctx2.tune_entries()) == sorted(ents)
        assert not compare(run(ctx2, b, "wfa", w["pen"], -1, dev=(dev, enc)), want)
    rng = np.random.default_rng(8)
    for i in rng.choice(b.n, 30, replace=False):
        st, sc, runs, _ = oracle.wfa_pair(b.pattern(i), b.text(i), w["pen"])
        assert (want[1][i], want[0][i]) == (st, sc) and want[2][want[3][i]:want[3][i + 1]].tolist() == runs, i


def test_graph_outlives_its_context():
    # a graph destroyed after its context (as Python may do) frees its HIP
    # objects without touching the context, and a launch of it is refused;
    # the next context works
    w = synth.WORKLOADS["swg150"]
    b = synth.workload("swg150", n=500)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        ctx = aim.Context(0)
        g, dev, outs, max_len, enc = _capture(ctx, b, w, stream)
        ctx.close()
        with pytest.raises(aim.AimError):
            g.launch(stream)
        g.close()
    with aim.Context(0) as c2:
        got = run(c2, b, w["alg"], w["pen"], w["max_score"], enc=w["enc"])
        assert not compare(got, oracle.align_batch(b, w["alg"], w["pen"], w["max_score"]))
