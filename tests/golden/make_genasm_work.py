"""Write tests/golden/genasm_work.json: GenASM work totals of the GenASM
workloads, counted by the oracle (oracle/genasm.c's work counters) over every
pair: windows, status-vector updates the distance calculation needs,
traceback steps, and the accepted pairs.  Calls only the generators and the
oracle."""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
import oracle  # noqa: E402
import synth  # noqa: E402

CHUNK = 50_000


def totals(name):
    w = synth.WORKLOADS[name]
    tot = np.zeros(3, np.int64)
    accepted = 0
    bases = 0
    for start in range(0, w["total"], CHUNK):
        b = synth.workload(name, start=start, n=min(CHUNK, w["total"] - start))
        st = np.zeros((b.n, 3), np.int64)
        _, status, _, _ = oracle.genasm_batch(b, w["max_score"], want_cigar=False, stats=st)
        tot += st.sum(axis=0)
        accepted += int((status == 0).sum())
        bases += int(b.pat_len.sum()) + int(b.txt_len.sum())
    return {"pairs": w["total"], "accepted": accepted, "windows": int(tot[0]), "updates": int(tot[1]),
            "tb_steps": int(tot[2]), "bases": bases}


if __name__ == "__main__":
    names = sys.argv[1:] or [n for n, w in synth.WORKLOADS.items() if w["alg"] == "genasm"]
    path = os.path.join(HERE, "genasm_work.json")
    out = json.load(open(path)) if os.path.exists(path) else {}
    for name in names:
        t0 = time.time()
        out[name] = totals(name)
        print(name, out[name], "%.0f s" % (time.time() - t0), flush=True)
        with open(path, "w") as f:
            json.dump(out, f, indent=1, sort_keys=True)
            f.write("\n")
