"""The host planners run on worker threads when batches and observables are
planned (cfh_batch_create, cfh_ham_create).  This builds them with
ThreadSanitizer into a small driver that plans several inputs on six
threads at once and compares every thread's plans with a serial run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2602_09020_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not present")
def test_planners_are_race_free_on_threads(tmp_path):
    exe = str(tmp_path / "planner_threads")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=thread", "-pthread",
           "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
           os.path.join(ROOT, "tests", "planner_threads.cpp"), os.path.join(CSRC, "plan.cpp"),
           os.path.join(CSRC, "frame.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1:exitcode=66")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout + r.stderr)[-3000:]
    assert "0 of 36 differ" in r.stdout
