"""WFA-adaptive on the GPU (alg "wfa_adaptive", k_wfa_lds with the
reduction step) against the CPU adaptive oracle (oracle.wfa_batch with the
same parameters): scores, statuses and CIGARs element by element, the count
of dropped diagonals, thresholds, long and lopsided pairs, the re-run of
pairs whose runs outgrow their slot and the pool, and the input limits.
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


def _pairs(seed, n, lmin, lmax, rmax, unrelated=0.0, lopsided=0):
    rng = np.random.default_rng(seed)
    pats, txts = [], []
    for k in range(n):
        T = rng.integers(0, 4, int(rng.integers(lmin, lmax + 1))).astype(np.uint8)
        if rng.random() < unrelated:
            P = rng.integers(0, 4, int(rng.integers(lmin, lmax + 1))).astype(np.uint8)
        else:
            bb = synth.from_lists([T], [T])
            P, _ = synth.mutate(rng, bb.txt, bb.txt_off, [float(rng.uniform(0, rmax))])
        if lopsided and k % 3 == 0:
            cut = int(rng.integers(0, min(lopsided, len(P)) + 1))
            P = P[cut:] if k % 2 else P[:len(P) - cut]
        pats.append(P)
        txts.append(T)
    return synth.from_lists(pats, txts)


def check(ctx, b, pen, adaptive, max_score=-1):
    ctx.wfa_adaptive_params(*adaptive)
    got = run(ctx, b, "wfa_adaptive", pen, max_score)
    want = oracle.wfa_batch(b, pen, max_score, adaptive=adaptive)
    bad = compare(got, want)
    assert not bad, "%d mismatches, first: %s" % (len(bad), describe(b, bad[0], got, want))
    return got


@pytest.mark.parametrize("pen", [AFF, (0, 1, 0, 1), (0, 3, 4, 1), (0, 9, 1, 1)])
@pytest.mark.parametrize("adaptive", [(10, 50), (4, 5), (1, 0)])
def test_mixed_pairs(ctx, pen, adaptive):
    b = _pairs(11, 700, 0, 600, 0.25, unrelated=0.1, lopsided=80)
    check(ctx, b, pen, adaptive)


def test_exhaustive_tiny(ctx):
    seqs = [np.array(s, np.uint8) for L in range(4) for s in itertools.product(range(4), repeat=L)]
    pats, txts = zip(*[(p, t) for p in seqs for t in seqs])
    b = synth.from_lists(list(pats), list(txts))
    for pen in [AFF, (0, 1, 0, 1)]:
        check(ctx, b, pen, (1, 0))


def test_dropped_count_and_thresholds(ctx):
    b = _pairs(12, 500, 50, 800, 0.2)
    adaptive = (4, 5)
    check(ctx, b, AFF, adaptive)
    st = ctx.last_call_stats()
    want = sum(oracle.wfa_pair(b.pattern(i), b.text(i), AFF, want_cigar=False, adaptive=adaptive)[3]["dropped"]
               for i in range(b.n))
    assert want > 0 and st["wfa_adaptive_dropped"] == want
    for smax in [0, 40, 300]:
        check(ctx, b, AFF, adaptive, smax)


def test_long_pairs(ctx):
    b = _pairs(13, 60, 2000, 10000, 0.1, lopsided=300)
    check(ctx, b, AFF, (10, 50))


def test_identical_to_exact_when_nothing_drops(ctx):
    b = _pairs(14, 400, 0, 300, 0.15)
    ctx.wfa_adaptive_params(10 ** 6, 0)
    got = run(ctx, b, "wfa_adaptive", AFF)
    assert not compare(got, oracle.align_batch(b, "swg", AFF, -1))


def test_runs_beyond_slot_and_pool_are_rerun():
    # 800 pairs of 8-10 kbp at up to 25 % error reserve thousands of pool
    # words each: a 256 MiB scratch limit leaves a pool of 2^20, which they
    # exhaust, so some are re-aligned in place by the adaptive re-run
    b = _pairs(15, 800, 8000, 10000, 0.25)
    with aim.Context(0, scratch_limit=256 << 20) as c:
        check(c, b, AFF, (10, 50))
        assert c.last_call_stats()["cigar_reruns"] > 0


def test_limits(ctx):
    b = _pairs(16, 4, 100, 200, 0.05)
    with pytest.raises(aim.AimError) as ei:
        run(ctx, b, "wfa_adaptive", AFF, max_len=16001)
    assert ei.value.code == -2
    with pytest.raises(aim.AimError):
        ctx.wfa_adaptive_params(0, 5)
    ctx.wfa_adaptive_params(10, 50)


@pytest.mark.parametrize("name,n", [("wfa_adaptive_150", 4000), ("wfa_adaptive_1k", 800)])
def test_graph_replays(name, n):
    # the adaptive pass and its in-place re-run captured once; every replay,
    # with eager work between them, gives the adaptive oracle's results
    from gpu_util import to_device
    w = synth.WORKLOADS[name]
    b = synth.workload(name, n=n)
    L = int(max(b.pat_len.max(), b.txt_len.max()))
    want = oracle.wfa_batch(b, w["pen"], w["max_score"], adaptive=w["adaptive"])
    cap = int((b.pat_len.astype(np.int64) + b.txt_len + 1).sum()) + 1
    stream = torch.cuda.Stream()
    print("adaptive graph replays: %s, %d pairs" % (name, n), flush=True)
    with aim.Context(0) as c, torch.cuda.stream(stream):
        c.wfa_adaptive_params(*w["adaptive"])
        dev, enc = to_device(b, w["enc"])
        outs = (torch.empty(b.n, dtype=torch.int32, device="cuda"), torch.empty(b.n, dtype=torch.int8, device="cuda"),
                torch.empty(cap, dtype=torch.int32, device="cuda"),
                torch.empty(b.n + 1, dtype=torch.int64, device="cuda"))
        g = c.graph_capture(*dev, enc=enc, max_len=L, alg="wfa_adaptive", pen=w["pen"], max_score=w["max_score"],
                            score=outs[0], status=outs[1], cigar=outs[2], cigar_off=outs[3], stream=stream)
        for rep in range(3):
            for t in outs:
                t.zero_()  # eager work between replays
            stream.synchronize()
            g.launch(stream)
            stream.synchronize()
            s, st, cg, off = outs
            got = (s.cpu().numpy(), st.cpu().numpy(), cg.cpu().numpy().view(np.uint32), off.cpu().numpy())
            bad = compare(got, want)
            assert not bad, (rep, describe(b, bad[0], got, want))
        g.close()
