"""Write tests/golden/wfa_work.json: the wavefront work of every pair of the
WFA workloads, counted by the scalar wavefront oracle (oracle/wfa_scalar.c,
whose counters tests/test_oracle_wfa_work.py pins).

Per workload: the totals of cells (diagonals of every non-null wavefront,
s = 0 included), 32-base extension words and bases compared, and the same
split by the pair's extent e = max(-lo_min, hi_max + 1), the half-width of
the smallest window centred on diagonal 0 that holds all of its wavefronts
(a kernel that keeps a window of W = 2e diagonals takes exactly the pairs of
extent <= e).  With a threshold, each row also counts the pairs, cells and
words of the pairs the pre-alignment filter lets through (lower bound from
oracle.prefilter at most the threshold): the wavefront kernels see only
those.  The counts are penalty-scale free: dividing x, o and e by
their common divisor leaves the non-null wavefronts and their ranges as they
are.

For the WFA-adaptive workloads the counts are those of the adaptive oracle
(the reduced wavefronts).

Runs the oracle only (no GPU code); about 10 minutes on 8 cores:
    python tests/golden/make_wfa_work.py [workload ...]
"""
from __future__ import annotations

import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402
from oracle.prefilter import lower_bounds  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "wfa_work.json")
# extent buckets (upper bounds, inclusive); the last catches the rest
EDGES = [32, 64, 96, 128, 192, 256, 384, 512, 1024, 2048, 4096, 8192, 1 << 30]
CHUNK = 20_000


def count(name: str, threads: int) -> dict:
    w = synth.WORKLOADS[name]
    total = w["total"]
    nb = len(EDGES)
    keys = ("pairs", "accepted", "cells", "words", "compared", "pass_pairs", "pass_cells", "pass_words")
    agg = {k: np.zeros(nb, np.int64) for k in keys}
    t0 = time.time()
    for start in range(0, total, CHUNK):
        b = synth.workload(name, start=start, n=min(CHUNK, total - start))

        def one(i):
            st, sc, _, c = oracle.wfa_pair(b.pattern(i), b.text(i), w["pen"], w["max_score"], want_cigar=False,
                                           adaptive=w.get("adaptive"))
            ext = max(-c["lo_min"], c["hi_max"] + 1)
            return st, ext, c["cells"], c["words"], c["compared"]

        with ThreadPoolExecutor(threads) as ex:
            res = list(ex.map(one, range(b.n)))
        lb = lower_bounds(b, "wfa", w["pen"], nthreads=threads) if w["max_score"] >= 0 else None
        for i, (st, ext, cells, words, comp) in enumerate(res):
            k = int(np.searchsorted(EDGES, ext))
            agg["pairs"][k] += 1
            agg["accepted"][k] += st == 0
            agg["cells"][k] += cells
            agg["words"][k] += words
            agg["compared"][k] += comp
            if lb is None or lb[i] <= w["max_score"]:
                agg["pass_pairs"][k] += 1
                agg["pass_cells"][k] += cells
                agg["pass_words"][k] += words
        print("%s: %d/%d pairs, %.0f s" % (name, start + b.n, total, time.time() - t0), flush=True)
    return {
        "penalties": list(w["pen"]), "max_score": w["max_score"], "pairs": total,
        "accepted": int(agg["accepted"].sum()), "cells": int(agg["cells"].sum()),
        "words": int(agg["words"].sum()), "compared": int(agg["compared"].sum()),
        "by_extent": [[e if e < (1 << 30) else None] + [int(agg[c][k]) for c in keys if c != "compared"]
                      for k, e in enumerate(EDGES)],
        "by_extent_columns": ["extent_max", "pairs", "accepted", "cells", "words", "pass_pairs", "pass_cells",
                              "pass_words"],
    }


def main():
    names = sys.argv[1:] or ["wfa250", "wfa_mixed"]
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    data["_note"] = ("written by tests/golden/make_wfa_work.py from the scalar wavefront oracle; "
                     "cells include s = 0; extent = max(-lo_min, hi_max + 1)")
    for name in names:
        data[name] = count(name, os.cpu_count() or 1)
        json.dump(data, open(OUT, "w"), indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
