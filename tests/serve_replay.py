"""Open-loop replay of the seeded serving schedule through aim_server.

The schedule (synth.serving_schedule): Poisson arrivals at 2,000 requests/s
for 60 s; each request holds 1-4,096 pairs (log-uniform), reads of 100-1,000
bp, an error rate uniform in [1 %, 8 %] and an algorithm drawn from NW edit,
SWG 4/6/2 and WFA 4/6/2.

Request contents.  The full schedule holds about 6e7 pairs (65 GB of bases),
more than the host's generator makes in the schedule's 60 s.  The requests'
arrival times, sizes, algorithms and penalties follow the schedule exactly;
their pairs are drawn from pools generated up front, one per error-rate bin
(8 bins of 0.875 % over [1 %, 8 %], each generated at its midpoint rate,
lengths uniform in [100, 1,000]): request r takes a seeded contiguous range of
its bin's pool.  `request_pairs` is that mapping; the tests use it too.

Latency = completion - scheduled arrival (queueing and submission lateness
included): the submission time on the client's clock plus the server's own
submission-to-completion time, so that collecting results in arrival order
does not delay a request's stamp.
"""
from __future__ import annotations

import gc
import threading
import time

import numpy as np

BINS = 8
RMIN, RMAX = 0.01, 0.08
POOL_PAIRS = 65536
_pools = {}


def _pool(synth, k):
    if k not in _pools:
        rng = synth._chunk_rng(synth.SERVE["seed"] * 7 + 1000 + k, 2)
        rate = RMIN + (k + 0.5) * (RMAX - RMIN) / BINS
        lens = rng.integers(synth.SERVE["lmin"], synth.SERVE["lmax"] + 1, POOL_PAIRS)
        _pools[k] = synth._gen_chunk(rng, POOL_PAIRS, lens, np.full(POOL_PAIRS, rate), None)
    return _pools[k]


def request_pairs(synth, req):
    """The pairs of request `req`: a contiguous range of its rate bin's pool
    (numpy views: pat, pat_off[n+1], txt, txt_off[n+1], relative offsets)."""
    k = min(BINS - 1, max(0, int((req.rate - RMIN) / ((RMAX - RMIN) / BINS))))
    p = _pool(synth, k)
    n = req.n_pairs
    o = int((req.seed * 2654435761) % (POOL_PAIRS - n + 1))
    po = p.pat_off[o:o + n + 1]
    to = p.txt_off[o:o + n + 1]
    return synth.PairBatch(p.pat[po[0]:po[-1]], po - po[0], p.txt[to[0]:to[-1]], to - to[0])


def submit(srv, req, b):
    return srv.submit(req.alg, req.pen, -1, b.pat, b.pat_off[:-1], b.pat_len, b.txt, b.txt_off[:-1],
                      b.txt_len)


def replay(aim, synth, seconds, streams, log, max_batch=0):
    t0 = time.time()
    sched = [r for r in synth.serving_schedule() if r.t_arrival < seconds]
    for k in range(BINS):
        _pool(synth, k)
    log("serving: %d requests; pools of %d pairs x %d rate bins in %.1f s" % (len(sched), POOL_PAIRS, BINS,
                                                                            time.time() - t0))
    srv = aim.Server(0, n_streams=streams, budget_bytes=64 << 30, max_batch_pairs=max_batch)
    # start-up: every worker runs one batch of the merge cap at the longest
    # reads per algorithm, so no worker grows its buffers mid-schedule
    cap = max_batch or 65536
    rng = np.random.default_rng(7)
    big = synth._gen_chunk(rng, cap, np.full(cap, synth.SERVE["lmax"]), np.full(cap, RMAX), None)
    for alg, pen in sorted({(r.alg, r.pen) for r in sched}):
        ws = [srv.submit(alg, pen, -1, big.pat, big.pat_off[:-1], big.pat_len, big.txt, big.txt_off[:-1],
                         big.txt_len) for _ in range(streams)]
        for i in ws:
            srv.wait(i)
    log("serving: warmed %d workers with %d-pair batches" % (streams, cap))
    srv.reset_stats()
    n = len(sched)
    ids = [None] * n
    submitted = [0.0] * n
    server_us = [0.0] * n
    pairs = [0] * n
    start = time.perf_counter()

    def producer():
        for k, r in enumerate(sched):
            b = request_pairs(synth, r)
            now = time.perf_counter() - start
            if r.t_arrival > now:
                time.sleep(r.t_arrival - now)
            rid = submit(srv, r, b)
            submitted[k] = time.perf_counter() - start
            pairs[k] = b.n
            ids[k] = rid

    gc.collect()
    gc.disable()  # no collector pauses in the replay's threads
    th = threading.Thread(target=producer)
    th.start()
    k = 0
    last = time.perf_counter()
    while k < n:
        if ids[k] is None:
            time.sleep(0.0005)
            continue
        server_us[k] = srv.wait(ids[k])[4]
        k += 1
        if time.perf_counter() - last > 5:
            log("serving: %d/%d requests done at %.1f s" % (k, n, time.perf_counter() - start))
            last = time.perf_counter()
    th.join()
    wall = time.perf_counter() - start
    gc.enable()
    st = srv.stats()
    srv.close()
    lat = np.array([(submitted[k] - sched[k].t_arrival) * 1e6 + server_us[k] for k in range(n)])
    late = np.array([submitted[k] - sched[k].t_arrival for k in range(n)])
    by_alg = {}
    for a in ("nw", "swg", "wfa"):
        sel = np.array([r.alg == a for r in sched])
        if sel.any():
            by_alg[a] = {"p50_us": round(float(np.percentile(lat[sel], 50)), 1),
                         "p99_us": round(float(np.percentile(lat[sel], 99)), 1), "requests": int(sel.sum())}
    total_pairs = int(sum(pairs))
    return {
        "p50_us": round(float(np.percentile(lat, 50)), 1),
        "p99_us": round(float(np.percentile(lat, 99)), 1),
        "server_p50_us": round(st["p50_us"], 1), "server_p99_us": round(st["p99_us"], 1),
        "by_algorithm": by_alg,
        "pairs_per_s": round(total_pairs / wall, 1),
        "offered_pairs_per_s": round(total_pairs / seconds, 1),
        "requests": n, "pairs": total_pairs, "batches": st["batches"], "wall_s": round(wall, 2),
        "peak_bytes": st["peak_bytes"], "budget_bytes": st["budget_bytes"],
        "max_submit_lateness_ms": round(float(late.max()) * 1000, 2) if n else 0.0,
        "p99_submit_lateness_ms": round(float(np.percentile(late, 99)) * 1000, 2) if n else 0.0,
        "schedule": "Poisson 2,000 requests/s, first %.1f s of the 60 s schedule; 1-4096 pairs per request "
                    "(log-uniform), 100-1000 bp, 1-8 %% error (pairs from per-rate-bin pools), NW 0/1/0/1 | "
                    "SWG 4/6/2 | WFA 4/6/2, score + CIGAR, 64 GiB budget, %d streams" % (seconds, streams),
    }
