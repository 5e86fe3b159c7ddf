"""The serving scheduler (paper_2208_01243_amd/csrc/serve_sched.h) on the
host: tests/serve_sched_test.cpp built with g++ and run, once optimised and
once under ThreadSanitizer (which fails the run on any data race)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "serve_sched_test.cpp")
INC = os.path.join(ROOT, "paper_2208_01243_amd", "csrc")


def _build_and_run(tmp_path, flags, env=None):
    exe = str(tmp_path / "serve_sched_test")
    subprocess.run(["g++", "-std=c++17", "-g", "-pthread", "-I" + INC] + flags + [SRC, "-o", exe], check=True)
    res = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    return res


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_scheduler_rules(tmp_path):
    res = _build_and_run(tmp_path, ["-O2", "-Wall"])
    assert res.returncode == 0 and "OK" in res.stdout, res.stdout + res.stderr


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_scheduler_thread_sanitizer(tmp_path):
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 second_deadlock_stack=1")
    res = _build_and_run(tmp_path, ["-O1", "-fsanitize=thread"], env=env)
    assert "ThreadSanitizer" not in res.stderr, res.stderr[-4000:]
    assert res.returncode == 0 and "OK" in res.stdout, res.stdout + res.stderr[-2000:]
