"""Benchmark: batched pairwise alignment throughput on one MI355X.

Default workload (the configuration the headline metric is quoted on):
Gotoh/SWG global alignment with penalties 4/6/2, 1,000,000 pairs of 150 bp
reads at 4 % error (1/3 each substitution, insertion, deletion), 2-bit packed
input, int32 scores and CIGARs.  One step = one aim_align_batch call over the
whole batch (input encoding, band tiers with exactness certificate, full-matrix
fallback, traceback, CIGAR compaction), inputs already resident in HBM.

Prints ONE JSON line.  Roofline: the dominant kernel is the 32-diagonal band
kernel; its duration comes from HIP events recorded on the launch stream around
every launch during the timed steps.  The CPU baseline is the oracle on a
bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_INT32_TOPS = 256 * 64 * 2.4e9 / 1e12  # 256 CUs x 64 lanes x 2.4 GHz = 39.3 T int32 ops/s
PEAK_PK16_TOPS = 2 * PEAK_INT32_TOPS       # packed 16-bit: two halves per lane = 78.6 T ops/s
HBM_PEAK_GBS = 8000.0
# algorithmic integer ops per DP cell (fill recurrences + traceback code):
# Gotoh: E 3, F 3, H 3 (diag add, two mins), 4 traceback bits 4 -> 13 (+1 for the
# mismatch test) = 14; linear NW: 2 adds + 2 mins + diag add + 2 bits + test = 10
OPS_PER_CELL = {"swg": 14, "nw": 10, "wfa": 14}
# HBM bytes per launch of the dominant kernel from two rocprofv3 --pmc passes
# (FETCH_SIZE x 2.0, WRITE_SIZE x 1.0 after the copy-kernel calibration; see
# profiles/k_band16_swg150_hbm_counters.md), valid only for the kernel source
# they were taken on (first 16 hex of its SHA-256).
MEASURED_TRAFFIC = {("swg150", "k_band16<32>"): ("32a97daf6917c56a", 3.0790e9)}

WORKLOAD_TEXT = {
    "swg150": "Gotoh 4/6/2 global, 1,000,000 pairs x 150 bp, 4% error (1/3 sub, ins, del), "
              "2-bit packed, int32 score + CIGAR",
    "nw100": "NW edit distance, 10,000 pairs x 100 bp, 2% error, threshold 5, uint8 ASCII, "
             "int32 score + CIGAR",
    "wfa250": "WFA 4/6/2, 1,000,000 pairs x 250 bp, 80% at 5% error + 20% unrelated, "
              "threshold 200, 2-bit, score + CIGAR",
    "wfa_mixed": "WFA 4/6/2, 500,000 pairs, 100-10,000 bp log-uniform, 0.5-10% error, 2-bit",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="swg150", choices=sorted(WORKLOAD_TEXT))
    ap.add_argument("--pairs", type=int, default=None, help="override the pair count")
    ap.add_argument("--plain-steps", type=int, default=2, help="steps of the plain kernel (0: skip)")
    ap.add_argument("--cpu-sample", type=int, default=200_000, help="pairs for the CPU baseline (0: skip)")
    ap.add_argument("--cpu-threads", type=int, default=16)
    ap.add_argument("--graph", action="store_true", help="time replays of a captured HIP graph")
    ap.add_argument("--serve", action="store_true",
                    help="serving form: Poisson request schedule through aim_server (own JSON line)")
    ap.add_argument("--serve-seconds", type=float, default=3.0,
                    help="seconds of the 60 s arrival schedule to replay")
    ap.add_argument("--serve-streams", type=int, default=4)
    ap.add_argument("--serve-max-batch", type=int, default=0,
                    help="serving form: most pairs merged into one device batch (0: library default)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a 1 GiB device-to-device copy (HBM counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(pairs are independent; sharding is described in DESIGN.md). Run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    if args.calibrate_copy:
        x = torch.ones(1 << 28, dtype=torch.int32, device="cuda")  # 1 GiB
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        log("copied 3 x 1 GiB")
        return
    import synth
    import paper_2208_01243_amd as aim
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from gpu_util import to_device

    if args.serve:
        serve_bench(args, aim, synth)
        return

    w = synth.WORKLOADS[args.workload]
    n_total = args.pairs or w["total"]
    t0 = time.time()
    batch = synth.workload(args.workload, n=n_total)
    log("generated %d pairs in %.1fs" % (batch.n, time.time() - t0))
    dev, enc = to_device(batch, w["enc"])
    n = batch.n
    max_len = int(max(batch.pat_len.max(), batch.txt_len.max()))
    cells_matrix = float((batch.pat_len.astype(np.float64) * batch.txt_len).sum())

    score = torch.empty(n, dtype=torch.int32, device="cuda")
    status = torch.empty(n, dtype=torch.int8, device="cuda")
    cap = int((batch.pat_len.astype(np.int64) + batch.txt_len + 1).sum() // 4) + 1024
    cigar = torch.empty(cap, dtype=torch.int32, device="cuda")
    cigar_off = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    stream = torch.cuda.current_stream()
    step = None

    def c_step(ctx):
        ctx.align_batch(*dev, enc=enc, max_len=max_len, alg=w["alg"], pen=w["pen"],
                        max_score=w["max_score"], score=score, status=status, cigar=cigar,
                        cigar_off=cigar_off, want_cigar=True, stream=stream)

    step = c_step
    ctx = aim.Context(0, timing=not args.graph)
    graph = None
    if args.graph:
        stream = torch.cuda.Stream()
        torch.cuda.set_stream(stream)
        graph = ctx.graph_capture(*dev, enc=enc, max_len=max_len, alg=w["alg"], pen=w["pen"],
                                  max_score=w["max_score"], score=score, status=status, cigar=cigar,
                                  cigar_off=cigar_off, want_cigar=True, stream=stream)
        step = lambda c: graph.launch(stream) if c is ctx else c_step(c)  # noqa: E731
    for k in range(args.warmup):
        t1 = time.perf_counter()
        step(ctx)
        torch.cuda.synchronize()
        log("warmup step %d: %.1f ms" % (k, (time.perf_counter() - t1) * 1000))
    ctx.timing_reset()
    torch.cuda.synchronize()
    elapsed_hint_ms = (time.perf_counter() - t1) * 1000 if args.warmup else 1e9
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(ctx)
        if elapsed_hint_ms > 20000:  # long workloads: show progress (syncs each step)
            torch.cuda.synchronize()
            log("step %d done at %.1f s" % (k, time.perf_counter() - t0))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    phases = ctx.timing()
    ms_per_step = elapsed * 1000.0 / args.steps
    st = status.cpu().numpy()
    aligned = int((st == 0).sum())
    rejected = int((st == 1).sum())
    pairs_per_s = n / (elapsed / args.steps)
    log("phases (ms per step): " + ", ".join("%s %.3f" % (k, v[0] / args.steps) for k, v in phases.items()))

    # roofline of the dominant kernel
    roof = None
    if w["alg"] in ("swg", "nw"):
        # dominant kernel: the first band tier (packed 16-bit when the value
        # bound allows, else 32-bit)
        kname, phase, peak, unit = ("k_band16<32>", "band16", PEAK_PK16_TOPS, "Tops/s (packed int16)") \
            if "band16" in phases else ("k_band<32>", "band32", PEAK_INT32_TOPS, "Tops/s (int32)")
        band_ms, band_launches = phases.get(phase, (0.0, 0))
        # algorithmic cells of the 32-diagonal band: every pair's rows x 32
        m = batch.pat_len.astype(np.int64)
        cells_band = float((m * 32).sum())
        ops = OPS_PER_CELL[w["alg"]] * cells_band
        if band_launches:
            t_launch = band_ms / band_launches / 1000.0
            achieved = ops / t_launch / 1e12
            import hashlib
            src_name = "dp_band16.hip" if phase == "band16" else "dp_band.hip"
            src = open(os.path.join(ROOT, "paper_2208_01243_amd", "csrc", src_name), "rb").read()
            h = hashlib.sha256(src).hexdigest()[:16]
            meas = MEASURED_TRAFFIC.get((args.workload, kname))
            traffic = meas[1] if (meas and meas[0] == h and n == w["total"]) else None
            roof = {"bound": "alu", "kernel": kname, "achieved": round(achieved, 3),
                    "peak": round(peak, 1), "unit": unit,
                    "frac": round(achieved / peak, 4), "traffic": traffic,
                    "avg_launch_ms": round(band_ms / band_launches, 4),
                    "ops_per_cell": OPS_PER_CELL[w["alg"]], "cells_per_launch": cells_band}
    else:
        # WFA: the dominant score pass (one wavefront per pair with its fused
        # walk, or the HBM-ring pass for pairs too wide for its window); the
        # wavefront cell count is not known without the scalar WFA, so the
        # fraction of peak comes from the SQ counters in profiles/ instead
        names = {"wfa_score": "k_wfa_score16", "wfa_score_hbm": "k_wfa_score"}
        ph = max((k for k in names if k in phases), key=lambda k: phases[k][0], default=None)
        if ph:
            wfa_ms, wfa_launches = phases[ph]
            roof = {"bound": "alu", "kernel": names[ph], "avg_launch_ms": round(wfa_ms / max(wfa_launches, 1), 4),
                    "achieved": None, "peak": round(PEAK_INT32_TOPS, 1), "unit": "Tops/s (int32)",
                    "frac": None, "traffic": None}

    # plain one-pair-per-workgroup kernel on the same pairs
    plain = None
    if args.plain_steps > 0:
        pctx = aim.Context(0, kernel="plain")
        step(pctx)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.plain_steps):
            step(pctx)
        torch.cuda.synchronize()
        pel = (time.perf_counter() - t0) / args.plain_steps
        plain = {"pairs_per_s": round(n / pel, 1), "ms_per_step": round(pel * 1000, 3),
                 "speedup_of_auto": round(pel / (elapsed / args.steps), 2)}
        pctx.close()
        # the production path must reproduce the plain kernel bit for bit
        s1, st1 = score.clone(), status.clone()
        step(ctx)
        torch.cuda.synchronize()
        assert torch.equal(s1, score) and torch.equal(st1, status)

    # CPU baseline: the oracle, on a bounded sample of the same workload
    cpu = None
    if args.cpu_sample > 0:
        import oracle
        k = min(args.cpu_sample, n)
        sub = synth.workload(args.workload, n=k)
        threads = max(1, min(args.cpu_threads, os.cpu_count() or 1))
        t0 = time.perf_counter()
        oracle.align_batch(sub, w["alg"], w["pen"], w["max_score"], nthreads=threads)
        ct = time.perf_counter() - t0
        cpu = {"value": round(k / ct, 1), "unit": "pairs/s", "cores": threads, "kind": "oracle",
               "sample": "first %d pairs of the same workload (full-matrix int32 %s + canonical "
                         "traceback, %.1f s wall)" % (k, "Gotoh" if w["alg"] != "nw" else "NW", ct)}

    out = {
        "metric": "aligned pairs/s + GCUPS at 1 MI355X",
        "value": round(pairs_per_s, 1),
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic (seeded generator standing in for the paper's read sets)",
        "config": {"workload": WORKLOAD_TEXT[args.workload], "pairs": n, "max_len": max_len,
                   "algorithm": w["alg"], "penalties": list(w["pen"]), "max_score": w["max_score"]},
        "aligned_pairs": aligned,
        "rejected_pairs": rejected,
        "gcups_matrix": round(cells_matrix / (elapsed / args.steps) / 1e9, 1),
        "phases_ms_per_step": {k: round(v[0] / args.steps, 4) for k, v in phases.items()},
        "roofline": roof,
        "plain_kernel": plain,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def serve_bench(args, aim, synth):
    """Open-loop replay of the seeded Poisson schedule (2,000 requests/s;
    1..4096 pairs per request, 100..1000 bp, 1..8 %, NW / SWG / WFA) through
    the serving loop; latency = completion minus scheduled arrival."""
    import threading
    sched = [r for r in synth.serving_schedule() if r.t_arrival < args.serve_seconds]
    t0 = time.time()
    batches = []
    for r in sched:
        b = synth.request_pairs(r)
        batches.append(b)
    log("generated %d requests, %d pairs in %.1fs" % (len(sched), sum(b.n for b in batches), time.time() - t0))
    srv = aim.Server(0, n_streams=args.serve_streams, budget_bytes=64 << 30,
                     max_batch_pairs=args.serve_max_batch)
    # warm every worker's context and kernels on one small request per algorithm
    warm = [srv.submit(r.alg, r.pen, -1, b.pat, b.pat_off[:-1], b.pat_len, b.txt, b.txt_off[:-1], b.txt_len)
            for r, b in list(zip(sched, batches))[:12]]
    for i in warm:
        srv.wait(i)
    # and with batches of the merge cap at the schedule's longest reads, one per
    # worker and algorithm, so that no worker grows its scratch mid-schedule
    # (a server pays this once at start-up)
    cap = args.serve_max_batch or 65536
    rng = np.random.default_rng(7)
    big = synth._gen_chunk(rng, cap, np.full(cap, 1000), np.full(cap, 0.08), None)
    for alg, pen in sorted({(r.alg, r.pen) for r in sched}):
        ws = [srv.submit(alg, pen, -1, big.pat, big.pat_off[:-1], big.pat_len, big.txt, big.txt_off[:-1],
                         big.txt_len) for _ in range(args.serve_streams)]
        for i in ws:
            srv.wait(i)
    log("warmed %d workers with %d-pair batches of 1000 bp" % (args.serve_streams, cap))
    srv.reset_stats()
    ids = [None] * len(sched)
    lateness = [0.0] * len(sched)
    submitted = [0.0] * len(sched)
    server_us = [0.0] * len(sched)
    start = time.perf_counter()

    def producer():
        for k, (r, b) in enumerate(zip(sched, batches)):
            now = time.perf_counter() - start
            if r.t_arrival > now:
                time.sleep(r.t_arrival - now)
            lateness[k] = time.perf_counter() - start - r.t_arrival
            rid = srv.submit(r.alg, r.pen, -1, b.pat, b.pat_off[:-1], b.pat_len, b.txt, b.txt_off[:-1],
                             b.txt_len)
            submitted[k] = time.perf_counter() - start
            ids[k] = rid

    # no collector pauses in the replay's threads while the schedule runs
    import gc
    gc.collect()
    gc.disable()
    th = threading.Thread(target=producer)
    th.start()
    k = 0
    last_log = time.perf_counter()
    while k < len(sched):
        if ids[k] is None:
            time.sleep(0.0005)
            continue
        # results are collected in arrival order, but each request's latency
        # is its own: submission (client clock) plus the server's submission
        # to completion time, so a slow request does not delay the later ones
        server_us[k] = srv.wait(ids[k])[4]
        k += 1
        if time.perf_counter() - last_log > 10:
            log("serving: %d/%d requests done" % (k, len(sched)))
            last_log = time.perf_counter()
    th.join()
    wall = time.perf_counter() - start
    gc.enable()
    st = srv.stats()
    srv.close()
    lat = np.array([(submitted[k] - sched[k].t_arrival) * 1e6 + server_us[k] for k in range(len(sched))])
    pairs = sum(b.n for b in batches)
    out = {
        "metric": "p50/p99 latency in serving loop (+ pairs/s)",
        "value": round(float(np.percentile(lat, 99)), 1),
        "unit": "us (p99, completion - scheduled arrival)",
        "higher_is_better": False,
        "n_gpus": 1,
        "p50_us": round(float(np.percentile(lat, 50)), 1),
        "p99_us": round(float(np.percentile(lat, 99)), 1),
        "server_p50_us": round(st["p50_us"], 1), "server_p99_us": round(st["p99_us"], 1),
        "pairs_per_s": round(pairs / wall, 1),
        "offered_pairs_per_s": round(pairs / args.serve_seconds, 1),
        "requests": len(sched), "pairs": pairs, "batches": st["batches"],
        "peak_bytes": st["peak_bytes"], "budget_bytes": st["budget_bytes"],
        "max_submit_lateness_ms": round(max(lateness) * 1000, 2),
        "data": "synthetic", "dtype": "int32",
        "config": {"workload": "Poisson 2,000 requests/s, first %.1f s of the 60 s schedule; 1-4096 pairs "
                               "per request (log-uniform), 100-1000 bp, 1-8 %% error, NW 0/1/0/1 | SWG 4/6/2 | "
                               "WFA 4/6/2, score + CIGAR, 64 GiB budget, %d streams"
                               % (args.serve_seconds, args.serve_streams)},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
