"""Serving form: continuous batching of requests of mixed sizes and
algorithms.  Each request's results must equal the oracle's and the same
request aligned alone; admission must keep the device footprint under the
budget without dropping or starving anyone."""
import threading

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
import synth  # noqa: E402
import paper_2208_01243_amd as aim  # noqa: E402
from gpu_util import compare, run  # noqa: E402

ALGS = [("nw", (0, 1, 0, 1), -1), ("swg", (0, 4, 6, 2), -1), ("wfa", (0, 4, 6, 2), -1),
        ("wfa", (0, 4, 6, 2), 60), ("nw", (0, 1, 0, 1), 8)]


def _requests(seed, count, lmax=400):
    rng = np.random.default_rng(seed)
    out = []
    for r in range(count):
        alg, pen, smax = ALGS[int(rng.integers(0, len(ALGS)))]
        n = int(synth.log_uniform_int(rng, 1, 300, 1)[0])
        lens = rng.integers(0, lmax + 1, n)
        txts = [rng.integers(0, 4, int(L)).astype(np.uint8) for L in lens]
        pats = []
        for T in txts:
            bb = synth.from_lists([T], [T])
            P, _ = synth.mutate(rng, bb.txt, bb.txt_off, [float(rng.uniform(0.0, 0.1))])
            pats.append(P)
        out.append((alg, pen, smax, synth.from_lists(pats, txts)))
    return out


def _submit(srv, alg, pen, smax, b, enc="code"):
    data = (lambda c: synth.ascii_from_codes(c)) if enc == "ascii" else (lambda c: c)
    return srv.submit(alg, pen, smax, data(b.pat), b.pat_off[:-1], b.pat_len, data(b.txt), b.txt_off[:-1],
                      b.txt_len, enc=aim.ENC_ASCII if enc == "ascii" else aim.ENC_CODE)


def test_mix_equals_alone_and_oracle():
    reqs = _requests(1, 60)
    with aim.Server(0, n_streams=4) as srv:
        ids = [_submit(srv, a, p, s, b, enc="ascii" if k % 2 else "code") for k, (a, p, s, b) in enumerate(reqs)]
        results = [srv.wait(i) for i in ids]
        st = srv.stats()
    assert st["completed"] == 60 and st["p99_us"] >= st["p50_us"] > 0
    with aim.Context(0) as ctx:
        for (alg, pen, smax, b), res in zip(reqs, results):
            got = res[:4]
            want = oracle.align_batch(b, alg, pen, smax)
            assert not compare(got, want)
            alone = run(ctx, b, alg, pen, smax, enc="code")
            assert not compare(got, alone)


def _long_requests(seed, count, n, L):
    rng = np.random.default_rng(seed)
    out = []
    for r in range(count):
        txts = [rng.integers(0, 4, int(rng.integers(L // 2, L + 1))).astype(np.uint8) for _ in range(n)]
        pats = []
        for T in txts:
            bb = synth.from_lists([T], [T])
            P, _ = synth.mutate(rng, bb.txt, bb.txt_off, [float(rng.uniform(0.0, 0.08))])
            pats.append(P)
        alg, pen = [("wfa", (0, 4, 6, 2)), ("swg", (0, 4, 6, 2)), ("nw", (0, 1, 0, 1))][r % 3]
        out.append((alg, pen, -1, synth.from_lists(pats, txts)))
    return out


def test_budget_bounds_device_memory_and_no_starvation():
    # two streams of 96 MiB each: requests queue behind the two workers, the
    # device memory the server holds (staging plus each context's scratch,
    # from the library's own accounting) stays within the budget, and every
    # request completes with the oracle's results
    reqs = _requests(2, 40, lmax=300) + _long_requests(9, 3, 600, 1000)
    budget = 2 * (96 << 20)
    with aim.Server(0, n_streams=2, budget_bytes=budget) as srv:
        ids = [_submit(srv, a, p, s, b) for a, p, s, b in reqs]
        queued = srv.stats()["queued"]
        results = [srv.wait(i) for i in ids]
        st = srv.stats()
    print("budget %d: peak %d, in use %d, queued after submit %d, batches %d" % (
        budget, st["peak_bytes"], st["bytes_in_use"], queued, st["batches"]), flush=True)
    assert 0 < st["peak_bytes"] <= budget and st["completed"] == len(reqs)
    assert 0 < st["bytes_in_use"] <= st["peak_bytes"]
    for (alg, pen, smax, b), res in zip(reqs, results):
        assert not compare(res[:4], oracle.align_batch(b, alg, pen, smax))


def test_oversized_request_and_budget_refused():
    # 64 MiB for one stream: 8 MiB of input staging, which 60,000 pairs of
    # 150 bp do not fit
    b = synth.workload("swg150", n=60000)
    with aim.Server(0, n_streams=1, budget_bytes=64 << 20) as srv:
        with pytest.raises(aim.AimError) as ei:
            _submit(srv, "swg", (0, 4, 6, 2), -1, b)
        assert ei.value.code == -1
        # a request that fits is still served
        small = synth.workload("swg150", n=500)
        assert not compare(srv.wait(_submit(srv, "swg", (0, 4, 6, 2), -1, small))[:4],
                           oracle.align_batch(small, "swg", (0, 4, 6, 2), -1))
    with pytest.raises(aim.AimError) as ei:
        aim.Server(0, n_streams=2, budget_bytes=100 << 20)  # under 64 MiB per stream
    assert ei.value.code == -1


def test_concurrent_submitters():
    reqs = _requests(3, 48, lmax=250)
    ids = [None] * len(reqs)
    with aim.Server(0, n_streams=4) as srv:
        def sub(k0):
            for k in range(k0, len(reqs), 4):
                a, p, s, b = reqs[k]
                ids[k] = _submit(srv, a, p, s, b)
        th = [threading.Thread(target=sub, args=(k,)) for k in range(4)]
        for t in th:
            t.start()
        for t in th:
            t.join()
        for (alg, pen, smax, b), i in zip(reqs, ids):
            assert not compare(srv.wait(i)[:4], oracle.align_batch(b, alg, pen, smax))


def test_schedule_distribution_mix_alone_and_oracle():
    # The serving schedule's own request distribution (1-4096 pairs, 100-1000
    # bp, 1-8 %, NW / SWG / WFA): the requests arriving in its first 0.25 s,
    # submitted together (the mix), then every one of them again alone; a
    # seeded 1 % of them (at least 5) is also checked against the oracle.
    import serve_replay
    sched = [r for r in synth.serving_schedule() if r.t_arrival < 0.25]
    batches = [serve_replay.request_pairs(synth, r) for r in sched]
    print("schedule check: %d requests, %d pairs" % (len(sched), sum(b.n for b in batches)), flush=True)
    with aim.Server(0, n_streams=4) as srv:
        ids = [serve_replay.submit(srv, r, b) for r, b in zip(sched, batches)]
        mix = [srv.wait(i)[:4] for i in ids]
        for k, (r, b) in enumerate(zip(sched, batches)):
            alone = srv.wait(serve_replay.submit(srv, r, b))[:4]
            assert not compare(mix[k], alone), k
    rng = np.random.default_rng(55)
    pick = rng.choice(len(sched), size=max(5, len(sched) // 100), replace=False)
    for k in pick:
        r, b = sched[k], batches[k]
        assert not compare(mix[k], oracle.align_batch(b, r.alg, r.pen, -1)), k
