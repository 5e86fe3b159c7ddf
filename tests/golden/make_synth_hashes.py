"""Write tests/golden/synth_sha256.json: SHA-256 of the first pairs of every
seeded workload and of the serving schedule.  Calls only the generators, so the
GPU machine and this machine can confirm they see identical inputs."""
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
import synth  # noqa: E402

N = 2048


def hashes():
    out = {name: synth.workload(name, n=N).sha256() for name in synth.WORKLOADS}
    sched = synth.serving_schedule()
    h = hashlib.sha256()
    for r in sched[:N]:
        h.update(repr((round(r.t_arrival, 9), r.alg, r.pen, round(r.rate, 12), r.n_pairs, r.seed)).encode())
    out["serving_schedule"] = h.hexdigest()
    out["serving_requests"] = len(sched)
    out["serving_first_request_pairs"] = synth.request_pairs(sched[0]).sha256()
    return out


if __name__ == "__main__":
    with open(os.path.join(HERE, "synth_sha256.json"), "w") as f:
        json.dump(hashes(), f, indent=1, sort_keys=True)
        f.write("\n")
