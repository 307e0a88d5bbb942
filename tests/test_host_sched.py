"""The request server's scheduler (csrc/sched.hpp, host code) against a fake
device: tests/host/sched_test.cpp built with g++ plainly, under the thread
sanitizer and under the address and undefined-behaviour sanitizers, and
run. No GPU: the scheduler's device side is an interface the test fakes."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "host", "sched_test.cpp")
INC = os.path.join(ROOT, "paper_1804_11174_amd", "csrc")

BUILDS = {
    "plain": ["-O2"],
    "tsan": ["-O1", "-g", "-fsanitize=thread"],
    "asan": ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"],
}


@pytest.mark.parametrize("name", list(BUILDS))
def test_scheduler_host(tmp_path, name):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no g++")
    exe = str(tmp_path / f"sched_{name}")
    cmd = [gxx, "-std=c++17", "-Wall", "-Wextra", "-pthread", "-I", INC, *BUILDS[name], SRC, "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1", ASAN_OPTIONS="detect_leaks=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "sched tests ok" in r.stdout
