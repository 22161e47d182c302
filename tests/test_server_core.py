"""The request loop's scheduling core on the CPU (no device): server_core.h driven by a simulated
executor (tests/server_core_test.cpp) -- per-map submission order under out-of-order completion,
batches of distinct maps and one precision, lone requests, the device-byte budget (first come,
first served), queue backpressure (EBUSY), refusals (over-budget, unknown map), and failures
injected at launch and at completion reported through poll.  Built with g++ under
AddressSanitizer + UndefinedBehaviorSanitizer, and again under ThreadSanitizer (worker threads
against submit / wait)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "server_core_test.cpp")
INC = os.path.join(ROOT, "paper_2408_09066_amd", "csrc")


def build_and_run(tmp_path, sanitize):
    gxx = shutil.which("g++")
    if not gxx:
        pytest.skip("g++ not available")
    exe = os.path.join(str(tmp_path), "server_core_" + sanitize.replace(",", "_"))
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", f"-fsanitize={sanitize}",
           "-I", INC, SRC, "-o", exe, "-pthread"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               TSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "all checks passed" in r.stdout


def test_scheduler_core_asan_ubsan(tmp_path):
    build_and_run(tmp_path, "address,undefined")


def test_scheduler_core_tsan(tmp_path):
    build_and_run(tmp_path, "thread")
