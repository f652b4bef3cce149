"""The QEQ server's host scheduler under sanitizers, on the CPU.

tests/native/sched_test.cpp drives the scheduler header the server is built
on (queue, footprint admission, slot threads, tickets) with a fake executor:
a mixed stream from several submitting and polling threads (results equal to
each request computed alone, budget and slot limits at every start, FIFO
admission), head-of-line blocking, the error paths (request above the
budget, unknown or repeated ticket, a failing executor, submit after stop,
stop and destruction with queued work). It is compiled twice, with
ThreadSanitizer and with AddressSanitizer + UndefinedBehaviorSanitizer, and
must run clean under both. The ThreadSanitizer build uses the ROCm LLVM
clang++: GCC 11's ThreadSanitizer runtime does not intercept
pthread_cond_clockwait, which libstdc++ uses for timed condition waits, and
then reports false double locks.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "native", "sched_test.cpp")
OUT = os.path.join(ROOT, "_build", "native")

CLANG = "/opt/rocm/lib/llvm/bin/clang++"
SANITIZERS = {
    "tsan": (CLANG, ["-fsanitize=thread"], {"TSAN_OPTIONS": "halt_on_error=1 second_deadlock_stack=1"}),
    "asan": ("g++", ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"],
             {"ASAN_OPTIONS": "detect_leaks=1 halt_on_error=1"}),
}


@pytest.mark.parametrize("san", sorted(SANITIZERS))
def test_scheduler_under_sanitizer(san):
    cxx, flags, env_extra = SANITIZERS[san]
    if shutil.which(cxx) is None:
        pytest.skip(f"{cxx} not available")
    os.makedirs(OUT, exist_ok=True)
    exe = os.path.join(OUT, f"sched_test_{san}")
    cmd = [cxx, "-std=c++17", "-O1", "-g", "-pthread", *flags,
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2503_21176_amd", "csrc"),
           SRC, "-o", exe]
    b = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert b.returncode == 0, b.stderr[-4000:]
    env = dict(os.environ, **env_extra)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, (r.stdout + r.stderr)[-6000:]
    assert "scheduler checks passed" in r.stdout
    assert "WARNING: ThreadSanitizer" not in r.stderr
    assert "ERROR: AddressSanitizer" not in r.stderr
