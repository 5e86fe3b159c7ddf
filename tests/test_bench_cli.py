"""bench.py's command-line contract on the CPU: one GPU only (more is refused
with a message and exit status 2, before anything touches a device), and the
measured-traffic table keyed on source files that exist."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BENCH = os.path.join(ROOT, "bench.py")


@pytest.mark.parametrize("argv,env", [(["--gpus", "2"], {}), (["--gpus", "8"], {}), ([], {"WORLD_SIZE": "2"})])
def test_more_than_one_gpu_is_refused(argv, env):
    e = dict(os.environ)
    e.update(env)
    r = subprocess.run([sys.executable, BENCH] + argv, capture_output=True, text=True, env=e, timeout=120)
    assert r.returncode == 2, r.stderr
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_table_names_existing_sources():
    sys.path.insert(0, ROOT)
    import bench
    csrc = os.path.join(ROOT, "paper_2208_01243_amd", "csrc")
    for (workload, kernel), (digest, nbytes) in bench.MEASURED_TRAFFIC.items():
        assert kernel in bench.KERNEL_SOURCE, kernel
        files = bench.KERNEL_SOURCE[kernel]
        assert files[0].endswith(".hip") and all(os.path.exists(os.path.join(csrc, f)) for f in files), files
        assert len(digest) == 16 and int(digest, 16) >= 0 and nbytes > 0
        assert len(bench.src_hash(kernel)) == 16
