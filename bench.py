"""Benchmark: batched pairwise alignment throughput on one MI355X.

Default workload (the largest single-GPU configuration): gap-affine WFA with
penalties 4/6/2, 500,000 pairs with read lengths log-uniform in
[100, 10,000] bp and error rates uniform in [0.5 %, 10 %], 2-bit packed
input, int32 scores and CIGARs, no threshold.  One step = one
aim_align_batch call over the whole batch (validation, length sort, the
wavefront passes with their fused CIGAR walks, the full-store fallback,
CIGAR compaction), inputs already resident in HBM.

Prints ONE JSON line.  Besides the headline it carries:
  roofline      -- the dominant kernel's algorithmic integer ops per launch
                   (wavefront cells x 8 + 32-base extension words x 10, the
                   cells of the pairs that launch completes, from
                   tests/golden/wfa_work.json) over its average launch time,
                   measured with HIP events on its launch stream;
  plain_kernel  -- the same pairs through the plain one-pair-per-workgroup
                   kernel (identical results are asserted);
  end_to_end    -- the rate with the host<->device transfers included;
  cpu_baseline  -- the oracle, built -O3 -march=native on this host, on a
                   bounded sample, on all granted cores and on one core;
  other_configs -- the NW edit (10k x 100 bp), SWG (1M x 150 bp) and WFA
                   (1M x 250 bp with 20 % unrelated pairs) workloads,
                   WFA-adaptive at 150 bp / 2 %, 1 kbp / 5 %, 10 kbp / 5 %,
                   and GenASM at 150 bp / 4 % (k 15) and 1 kbp / 5 % (k 100);
  serving       -- the Poisson request schedule through aim_server.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_INT32_TOPS = 256 * 64 * 2.4e9 / 1e12  # 256 CUs x 64 lanes x 2.4 GHz = 39.3 T int32 ops/s
PEAK_PK16_TOPS = 2 * PEAK_INT32_TOPS       # packed 16-bit: two halves per lane = 78.6 T ops/s
# algorithmic integer ops per unit: a DP cell (fill recurrences + traceback
# code; Gotoh 14, linear NW 10), a wavefront cell (I, D, X candidates with
# their bounds, the max of M: 8) and a 32-base extension word (load, align,
# xor, count trailing zeros, advance: 10)
OPS_PER_CELL = {"swg": 14, "nw": 10}
WFA_OPS_PER_CELL, WFA_OPS_PER_WORD = 8, 10
# GenASM: a status-vector update (one 64-bit vector at one text position and
# edit level: match shift, start bit and text mask; the level below's
# substitution, insertion and deletion terms; the window mask: 14 int32 ops)
# stores its 8-byte vector for the traceback; a traceback step (12 ops) reads
# at least one stored vector
GENASM_OPS_PER_UPDATE, GENASM_OPS_PER_STEP, GENASM_BYTES_PER_UPDATE, GENASM_BYTES_PER_STEP = 14, 12, 8, 8
PEAK_HBM_GBS = 8000.0
# HBM bytes per launch of a kernel from two rocprofv3 --pmc passes (FETCH_SIZE
# and WRITE_SIZE scaled by a copy-kernel calibration), valid only for the
# kernel source they were taken on (first 16 hex of the SHA-256 of its source
# file and the headers it includes)
MEASURED_TRAFFIC = {("swg150", "k_band16<32>"): ("493d99bad8e4c2d4", 3.0799e9),
                    ("wfa_mixed", "k_wfa_lds"): ("40348926033b3dc9", 2.2745e12),
                    ("wfa250", "k_wfa_score16"): ("04f13bb9e7d35d4f", 4.335e9),
                    ("genasm150", "k_genasm"): ("4e069b03afdd5683", 5.15e9)}
KERNEL_SOURCE = {"k_band16<32>": ("dp_band16.hip", "aim_internal.h", "dev_util.h"),
                 "k_band<32>": ("dp_band.hip", "aim_internal.h"),
                 "k_wfa_score16": ("wfa.hip", "aim_internal.h", "wfa_common.h"),
                 "k_wfa_score": ("wfa.hip", "aim_internal.h", "wfa_common.h"),
                 "k_wfa_lds": ("wfa_lds.hip", "aim_internal.h", "wfa_common.h"),
                 "k_genasm": ("genasm.hip", "aim_internal.h", "dev_util.h")}

WORKLOAD_TEXT = {
    "swg150": "Gotoh 4/6/2 global, 1,000,000 pairs x 150 bp, 4% error (1/3 sub, ins, del), "
              "2-bit packed, int32 score + CIGAR",
    "nw100": "NW edit distance, 10,000 pairs x 100 bp, 2% error, threshold 5, uint8 ASCII, "
             "int32 score + CIGAR",
    "wfa250": "WFA 4/6/2, 1,000,000 pairs x 250 bp, 80% at 5% error + 20% unrelated, "
              "threshold 200, 2-bit, score + CIGAR",
    "wfa_mixed": "WFA 4/6/2, 500,000 pairs, 100-10,000 bp log-uniform, 0.5-10% error, 2-bit, "
                 "score + CIGAR",
    "wfa_adaptive_150": "WFA-adaptive 4/6/2 (10, 50), 1,000,000 pairs x 150 bp, 2% error, 2-bit, score + CIGAR",
    "wfa_adaptive_1k": "WFA-adaptive 4/6/2 (10, 50), 100,000 pairs x 1,000 bp, 5% error, 2-bit, score + CIGAR",
    "wfa_adaptive_10k": "WFA-adaptive 4/6/2 (10, 50), 10,000 pairs x 10,000 bp, 5% error, 2-bit, "
                        "score + CIGAR",
    "genasm150": "GenASM (windows of 64, overlap 24), k = 15 edits, 1,000,000 pairs x 150 bp, 4% error, "
                 "2-bit, score + CIGAR",
    "genasm1k": "GenASM (windows of 64, overlap 24), k = 100 edits, 100,000 pairs x 1,000 bp, 5% error, "
                "2-bit, score + CIGAR",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def src_hash(kernel):
    """The kernel's source file and the headers it includes, hashed together."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCE[kernel]:
        h.update(open(os.path.join(ROOT, "paper_2208_01243_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def genasm_units(name):
    """GenASM work totals of a whole workload from the oracle's counters
    (tests/golden/genasm_work.json), or None."""
    path = os.path.join(ROOT, "tests", "golden", "genasm_work.json")
    if not os.path.exists(path):
        return None
    return json.load(open(path)).get(name)


def wfa_units(name, window, filtered=False):
    """(cells, words) of the pairs the one-wavefront pass completes (extent <=
    window / 2) and of the rest, from the oracle's counts; None if absent.
    filtered: only the pairs the pre-alignment filter lets through (the
    wavefront kernels see no others)."""
    path = os.path.join(ROOT, "tests", "golden", "wfa_work.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path)).get(name)
    if not d:
        return None
    cols = d["by_extent_columns"]
    ci, wi = cols.index("pass_cells" if filtered else "cells"), cols.index("pass_words" if filtered else "words")
    inside = [0, 0]
    outside = [0, 0]
    for row in d["by_extent"]:
        ext_max = row[0]
        tgt = inside if (ext_max is not None and ext_max <= window // 2) else outside
        tgt[0] += row[ci]
        tgt[1] += row[wi]
    return {"inside": inside, "outside": outside, "cells": inside[0] + outside[0], "words": inside[1] + outside[1]}


class Run:
    """A workload on the device with its outputs, and one aligning step."""

    def __init__(self, aim, synth, name, n=None):
        import torch
        from gpu_util import to_device
        self.torch = torch
        self.name = name
        self.w = synth.WORKLOADS[name]
        self.n_total = n or self.w["total"]
        t0 = time.time()
        self.batch = synth.workload(name, n=self.n_total)
        b = self.batch
        self.dev, self.enc = to_device(b, self.w["enc"])
        log("%s: generated and moved %d pairs in %.1f s" % (name, b.n, time.time() - t0))
        self.n = b.n
        self.max_len = int(max(b.pat_len.max(), b.txt_len.max()))
        self.cells_matrix = float((b.pat_len.astype(np.float64) * b.txt_len).sum())
        self.score = torch.empty(self.n, dtype=torch.int32, device="cuda")
        self.status = torch.empty(self.n, dtype=torch.int8, device="cuda")
        cap = int((b.pat_len.astype(np.int64) + b.txt_len + 1).sum() // 4) + 1024
        self.cigar = torch.empty(cap, dtype=torch.int32, device="cuda")
        self.cigar_off = torch.empty(self.n + 1, dtype=torch.int64, device="cuda")

    def step(self, ctx, stream=None):
        w = self.w
        ctx.align_batch(*self.dev, enc=self.enc, max_len=self.max_len, alg=w["alg"], pen=w["pen"],
                        max_score=w["max_score"], score=self.score, status=self.status, cigar=self.cigar,
                        cigar_off=self.cigar_off, want_cigar=True, stream=stream)

    def timed(self, ctx, steps, warmup):
        torch = self.torch
        for k in range(warmup):
            t1 = time.perf_counter()
            self.step(ctx)
            torch.cuda.synchronize()
            log("%s warmup %d: %.1f ms" % (self.name, k, (time.perf_counter() - t1) * 1000))
        ctx.timing_reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            self.step(ctx)
        torch.cuda.synchronize()
        return time.perf_counter() - t0


def roofline(run, phases, stats, steps):
    """Roofline of the dominant kernel (see the module docstring)."""
    w = run.w
    if w["alg"] in ("swg", "nw") and ("band16" in phases or "band32" in phases):
        kname, phase, peak, unit = ("k_band16<32>", "band16", PEAK_PK16_TOPS, "Tops/s (packed int16)") \
            if "band16" in phases else ("k_band<32>", "band32", PEAK_INT32_TOPS, "Tops/s (int32)")
        ms, launches = phases[phase]
        cells = float((run.batch.pat_len.astype(np.int64) * 32).sum())
        ops = OPS_PER_CELL[w["alg"]] * cells
        t = ms / launches / 1000.0
        meas = MEASURED_TRAFFIC.get((run.name, kname))
        traffic = meas[1] if (meas and meas[0] == src_hash(kname) and run.n == w["total"]) else None
        return {"bound": "alu", "kernel": kname, "achieved": round(ops / t / 1e12, 3), "peak": round(peak, 1),
                "unit": unit, "frac": round(ops / t / 1e12 / peak, 4), "traffic": traffic,
                "avg_launch_ms": round(ms / launches, 4), "ops_per_unit": OPS_PER_CELL[w["alg"]],
                "units_per_launch": cells, "unit_name": "band cells (m x 32 per pair)"}
    if w["alg"] == "wfa_adaptive":
        # one kernel (k_wfa_lds with the reduction step) over every pair
        if "wfa_adaptive" not in phases:
            return None
        ms, launches = phases["wfa_adaptive"]
        ms /= max(1, launches)
        units = wfa_units(run.name, 0) if run.n == w["total"] else None
        out = {"bound": "alu", "kernel": "k_wfa_lds (adaptive)", "avg_launch_ms": round(ms, 4),
               "peak": round(PEAK_INT32_TOPS, 1), "unit": "Tops/s (int32)",
               "ops_per_unit": {"wavefront cell": WFA_OPS_PER_CELL, "extension word": WFA_OPS_PER_WORD},
               "achieved": None, "frac": None, "traffic": None}
        if units:
            ops = WFA_OPS_PER_CELL * units["cells"] + WFA_OPS_PER_WORD * units["words"]
            out.update({"achieved": round(ops / (ms / 1000) / 1e12, 3),
                        "frac": round(ops / (ms / 1000) / 1e12 / PEAK_INT32_TOPS, 4),
                        "units_per_launch": {"cells": units["cells"], "words": units["words"]},
                        "unit_name": "cells of the reduced wavefronts (adaptive oracle) of every pair"})
        return out
    if w["alg"] == "genasm":
        # one kernel, k_genasm, over every pair: the distance calculation is
        # integer ALU work, and every status vector it builds is stored for
        # the traceback, so both rooflines are given; `bound` is the tighter
        if "genasm" not in phases:
            return None
        ms, launches = phases["genasm"]
        ms /= max(1, launches)
        u = genasm_units(run.name) if run.n == w["total"] else None
        meas = MEASURED_TRAFFIC.get((run.name, "k_genasm"))
        out = {"kernel": "k_genasm", "avg_launch_ms": round(ms, 4), "bound": "alu", "achieved": None,
               "peak": round(PEAK_INT32_TOPS, 1), "unit": "Tops/s (int32)", "frac": None, "traffic": None,
               "ops_per_unit": {"status-vector update": GENASM_OPS_PER_UPDATE,
                                "traceback step": GENASM_OPS_PER_STEP},
               "bytes_per_unit": {"status-vector update": GENASM_BYTES_PER_UPDATE,
                                  "traceback step": GENASM_BYTES_PER_STEP, "base": 0.25}}
        if u:
            t = ms / 1000.0
            ops = GENASM_OPS_PER_UPDATE * u["updates"] + GENASM_OPS_PER_STEP * u["tb_steps"]
            byts = GENASM_BYTES_PER_UPDATE * u["updates"] + GENASM_BYTES_PER_STEP * u["tb_steps"] + u["bases"] / 4
            alu = {"achieved": round(ops / t / 1e12, 3), "peak": round(PEAK_INT32_TOPS, 1), "unit": "Tops/s (int32)",
                   "frac": round(ops / t / 1e12 / PEAK_INT32_TOPS, 4)}
            hbm = {"achieved": round(byts / t / 1e9, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                   "frac": round(byts / t / 1e9 / PEAK_HBM_GBS, 4)}
            top = hbm if hbm["frac"] > alu["frac"] else alu
            out.update(top)
            out["bound"] = "hbm" if top is hbm else "alu"
            if meas and meas[0] == src_hash("k_genasm"):
                out["traffic"] = meas[1]
            out.update({"alu": alu, "hbm": hbm,
                        "units_per_launch": {"updates": u["updates"], "tb_steps": u["tb_steps"],
                                             "windows": u["windows"], "bases": u["bases"]},
                        "unit_name": "status-vector updates (distance + 1) x text bases per window and "
                                     "traceback steps, from the oracle's counters over every pair"})
        return out
    if w["alg"] != "wfa":
        return None
    # the WFA passes of one call: the one-wavefront pass (k_wfa_score16) over
    # every pair, completing those whose wavefronts stay in its window; the
    # window classes (k_wfa_lds, one launch per class, taken together: the
    # split of pairs between classes is a runtime prediction) completing the
    # rest; the HBM-ring pass (k_wfa_score) for pairs past 16,000 scores
    steps = max(1, phases.get("wfa_score", (0.0, 1))[1])
    groups = {"k_wfa_score16": ["wfa_score"], "k_wfa_lds": [k for k in phases if k.startswith("wfa_lds")],
              "k_wfa_score": ["wfa_score_hbm"]}
    per_call = {g: sum(phases[k][0] for k in ks if k in phases) / steps for g, ks in groups.items()}
    kname = max(per_call, key=per_call.get)
    if per_call[kname] <= 0:
        return None
    ms = per_call[kname]
    launches = sum(phases[k][1] for k in groups[kname] if k in phases) // steps
    filtered = w["max_score"] >= 0  # the pre-alignment filter runs in front
    units = wfa_units(run.name, stats.get("wfa_window", 0), filtered) if run.n == w["total"] else None
    out = {"bound": "alu", "kernel": kname, "avg_launch_ms": round(ms, 4), "launches_per_call": launches,
           "peak": round(PEAK_INT32_TOPS, 1), "unit": "Tops/s (int32)",
           "ops_per_unit": {"wavefront cell": WFA_OPS_PER_CELL, "extension word": WFA_OPS_PER_WORD},
           "achieved": None, "frac": None, "traffic": None}
    if units and kname != "k_wfa_score":
        side = "inside" if kname == "k_wfa_score16" else "outside"
        cells, words = units[side]
        ops = WFA_OPS_PER_CELL * cells + WFA_OPS_PER_WORD * words
        t = ms / 1000.0
        out.update({"achieved": round(ops / t / 1e12, 3), "frac": round(ops / t / 1e12 / PEAK_INT32_TOPS, 4),
                    "units_per_launch": {"cells": cells, "words": words},
                    "unit_name": "wavefront cells of the pairs %s completes (%s the %d-diagonal window%s), "
                                 "its launches of one call together" % (
                                     kname, side, stats.get("wfa_window", 0),
                                     "; pairs past the pre-alignment filter" if filtered else "")})
        meas = MEASURED_TRAFFIC.get((run.name, kname))
        if meas and meas[0] == src_hash(kname):
            out["traffic"] = meas[1]
        # every WFA kernel of the step together
        tot_ms = sum(v[0] for k, v in phases.items() if k.startswith("wfa")) / steps
        ops_all = WFA_OPS_PER_CELL * units["cells"] + WFA_OPS_PER_WORD * units["words"]
        out["all_wfa_kernels"] = {"ms_per_step": round(tot_ms, 3), "cells": units["cells"],
                                  "words": units["words"],
                                  "achieved": round(ops_all / (tot_ms / 1000) / 1e12, 3),
                                  "frac": round(ops_all / (tot_ms / 1000) / 1e12 / PEAK_INT32_TOPS, 4)}
    return out


def measure(aim, synth, name, steps, warmup, plain_steps=0, e2e_reps=0):
    import torch
    run = Run(aim, synth, name)
    ctx = aim.Context(0, timing=True)
    elapsed = run.timed(ctx, steps, warmup)
    phases = ctx.timing()
    stats = ctx.last_call_stats()
    ms_step = elapsed * 1000.0 / steps
    st = run.status.cpu().numpy()
    res = {"workload": WORKLOAD_TEXT[name], "pairs": run.n, "max_len": run.max_len,
           "pairs_per_s": round(run.n / (elapsed / steps), 1), "ms_per_step": round(ms_step, 4),
           "aligned_pairs": int((st == 0).sum()), "rejected_pairs": int((st == 1).sum()),
           "gcups_matrix": round(run.cells_matrix / (elapsed / steps) / 1e9, 1),
           "phases_ms_per_step": {k: round(v[0] / steps, 4) for k, v in phases.items()},
           "path_counters": stats}
    log("%s: %.3f ms/step; phases %s" % (name, ms_step, res["phases_ms_per_step"]))
    res["roofline"] = roofline(run, phases, stats, steps)
    units = wfa_units(name, 0) if run.w["alg"].startswith("wfa") and run.n == run.w["total"] else None
    if units:
        res["wavefront_cells_per_s"] = round(units["cells"] / (elapsed / steps), 1)
    if plain_steps > 0 and run.w["alg"] in ("nw", "swg", "wfa"):
        pctx = aim.Context(0, kernel="plain")
        s1, st1, off1 = run.score.clone(), run.status.clone(), run.cigar_off.clone()
        t0 = time.perf_counter()
        run.step(pctx)
        torch.cuda.synchronize()
        log("%s: plain warm-up step %.1f s" % (name, time.perf_counter() - t0))
        t0 = time.perf_counter()
        for _ in range(plain_steps):
            run.step(pctx)
        torch.cuda.synchronize()
        pel = (time.perf_counter() - t0) / plain_steps
        assert torch.equal(s1, run.score) and torch.equal(st1, run.status) and torch.equal(off1, run.cigar_off)
        pctx.close()
        res["plain_kernel"] = {"pairs_per_s": round(run.n / pel, 1), "ms_per_step": round(pel * 1000, 3),
                               "speedup_of_batched": round(pel / (elapsed / steps), 2),
                               "identical_results": True}
    if e2e_reps > 0:
        res["end_to_end"] = end_to_end(run, ctx, e2e_reps)
    ctx.close()
    return run, res


def end_to_end(run, ctx, reps):
    """Host pinned inputs -> H2D -> align -> D2H of scores, statuses, offsets
    and the CIGAR runs; median of `reps`."""
    torch = run.torch
    host = [t.cpu().pin_memory() for t in run.dev]
    h_score = torch.empty(run.n, dtype=torch.int32).pin_memory()
    h_status = torch.empty(run.n, dtype=torch.int8).pin_memory()
    h_off = torch.empty(run.n + 1, dtype=torch.int64).pin_memory()
    h_cig = torch.empty(run.cigar.numel(), dtype=torch.int32).pin_memory()
    times = []
    for _ in range(reps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for d, h in zip(run.dev, host):
            d.copy_(h, non_blocking=True)
        run.step(ctx)
        h_score.copy_(run.score, non_blocking=True)
        h_status.copy_(run.status, non_blocking=True)
        h_off.copy_(run.cigar_off, non_blocking=True)
        torch.cuda.synchronize()
        k = int(h_off[-1])
        h_cig[:k].copy_(run.cigar[:k], non_blocking=True)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    t = float(np.median(times[1:]))
    in_b = sum(h.numel() * h.element_size() for h in host)
    out_b = run.n * 13 + 4 * int(h_off[-1])
    return {"pairs_per_s": round(run.n / t, 1), "ms_per_step": round(t * 1000, 3),
            "bytes_in": in_b, "bytes_out": out_b, "reps": reps}


def cpu_baseline(synth, name, n_all, n_one):
    """The oracle on the first pairs of the workload: a -O3 -march=native build
    on this host, on all granted cores (at most 16: the CPU share of one GPU
    on the measurement boxes) and on one core; plus the scalar wavefront
    oracle for the WFA workloads."""
    import oracle
    w = synth.WORKLOADS[name]
    tmp = tempfile.mkdtemp(prefix="aim_oracle_")
    h = oracle.bind(oracle.build(path=os.path.join(tmp, "liboracle_native.so"), native=True))
    nproc = os.cpu_count() or 1
    threads = max(1, min(nproc, 16))
    out = {}
    for label, k, th in (("all", n_all, threads), ("one", n_one, 1)):
        sub = synth.workload(name, n=k)
        t0 = time.perf_counter()
        if w["alg"] == "genasm":
            oracle.genasm_batch(sub, w["max_score"], nthreads=th, handle=h)
        else:
            oracle.align_batch(sub, w["alg"], w["pen"], w["max_score"], nthreads=th, handle=h)
        ct = time.perf_counter() - t0
        out[label] = (k, th, ct)
        log("cpu oracle %s: %d pairs on %d threads in %.1f s" % (name, k, th, ct))
    k, th, ct = out["all"]
    k1, _, ct1 = out["one"]
    res = {"value": round(k / ct, 1), "unit": "pairs/s", "cores": th, "kind": "oracle",
           "host_nproc": nproc,
           "sample": "first %d pairs of the same workload: %s, gcc -O3 -march=native, %d threads, %.1f s wall" % (
                         k, {"nw": "full-matrix int32 NW + canonical traceback",
                             "genasm": "the plain windowed bitap + traceback (byte per bit, all k + 1 levels)"}.get(
                             w["alg"], "full-matrix int32 Gotoh + canonical traceback"), th, ct),
           "one_core": {"value": round(k1 / ct1, 1), "unit": "pairs/s", "cores": 1,
                        "sample": "first %d pairs, %.1f s" % (k1, ct1)}}
    if w["alg"] == "wfa":
        from concurrent.futures import ThreadPoolExecutor
        kw = min(10_000, w["total"])
        sub = synth.workload(name, n=kw)

        def one(i):
            return oracle.wfa_pair(sub.pattern(i), sub.text(i), w["pen"], w["max_score"], handle=h)[0]

        t0 = time.perf_counter()
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(one, range(sub.n)))
        ct = time.perf_counter() - t0
        res["scalar_wfa"] = {"value": round(kw / ct, 1), "unit": "pairs/s", "cores": threads,
                             "sample": "first %d pairs, the scalar wavefront oracle with CIGAR, %.1f s" % (kw, ct)}
        log("cpu scalar WFA: %d pairs in %.1f s" % (kw, ct))
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="wfa_mixed", choices=sorted(WORKLOAD_TEXT))
    ap.add_argument("--plain-steps", type=int, default=1, help="steps of the plain kernel (0: skip)")
    ap.add_argument("--e2e-reps", type=int, default=3, help="end-to-end reps with transfers (0: skip)")
    ap.add_argument("--cpu", type=int, default=1, help="CPU baseline (0: skip)")
    ap.add_argument("--others", type=int, default=1, help="also measure the other workloads (0: skip)")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="seconds of the serving schedule to replay (0: skip)")
    ap.add_argument("--serve-streams", type=int, default=4)
    ap.add_argument("--serve-only", action="store_true", help="only the serving replay (own JSON line)")
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
    import serve_replay

    if args.serve_only:
        print(json.dumps(serve_replay.replay(aim, synth, args.serve_seconds, args.serve_streams, log)), flush=True)
        return

    run, main_res = measure(aim, synth, args.workload, args.steps, args.warmup,
                            plain_steps=args.plain_steps, e2e_reps=args.e2e_reps)
    del run
    torch.cuda.empty_cache()
    w = synth.WORKLOADS[args.workload]
    out = {
        "metric": "aligned pairs/s + GCUPS at 1 MI355X",
        "value": main_res["pairs_per_s"],
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic (seeded generator standing in for the paper's read sets)",
        "config": {"workload": WORKLOAD_TEXT[args.workload], "pairs": main_res["pairs"],
                   "max_len": main_res["max_len"], "algorithm": w["alg"], "penalties": list(w["pen"]),
                   "max_score": w["max_score"]},
    }
    for k in ("aligned_pairs", "rejected_pairs", "gcups_matrix", "wavefront_cells_per_s", "phases_ms_per_step",
              "path_counters", "roofline", "plain_kernel", "end_to_end"):
        if k in main_res:
            out[k] = main_res[k]
    if args.cpu:
        n_all, n_one = {"wfa_mixed": (4000, 400), "swg150": (200_000, 20_000), "wfa250": (100_000, 10_000),
                        "nw100": (10_000, 10_000), "genasm150": (200_000, 20_000),
                        "genasm1k": (10_000, 1000)}.get(args.workload, (2000, 200))
        out["cpu_baseline"] = cpu_baseline(synth, args.workload, n_all, n_one)
    if args.others:
        others = {}
        for name in ("nw100", "swg150", "wfa250", "wfa_adaptive_150", "wfa_adaptive_1k", "wfa_adaptive_10k",
                     "genasm150", "genasm1k"):
            if name == args.workload:
                continue
            r, res = measure(aim, synth, name, 20, 3)
            del r
            torch.cuda.empty_cache()
            others[name] = {k: res[k] for k in ("workload", "pairs_per_s", "ms_per_step", "gcups_matrix",
                                                 "aligned_pairs", "rejected_pairs", "roofline",
                                                 "phases_ms_per_step", "path_counters")
                            if k in res}
        out["other_configs"] = others
    if args.serve_seconds > 0:
        # The serving replay runs in a process of its own, as a server does:
        # in this one, after the batch workloads, its latencies came out
        # ~40 % higher with the same schedule kept as closely -- and so they do
        # after allocating and freeing 100 GiB through torch alone, so it is
        # the state the device memory is left in, not the library.
        import subprocess
        cmd = [sys.executable, os.path.abspath(__file__), "--serve-only", "--serve-seconds",
               str(args.serve_seconds), "--serve-streams", str(args.serve_streams)]
        r = subprocess.run(cmd, stdout=subprocess.PIPE, text=True)
        if r.returncode != 0:
            log("serving replay failed with exit status %d" % r.returncode)
            sys.exit(1)
        out["serving"] = json.loads(r.stdout.strip().splitlines()[-1])
        out["serving"]["process"] = "own process (bench.py --serve-only)"
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
