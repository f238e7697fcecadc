"""The serving queue's host logic (csrc/queue.cpp, unchanged) built with g++ against a mock
executor and fake clock (tests/host_queue/), under the address + undefined-behaviour
sanitizers and under the thread sanitizer: admission by budget and slots, arrival order,
latency bookkeeping, release of finished tickets, the kernel-time union against the intervals
the executor recorded, and concurrent submitters (tests/host_queue/queue_check.cpp).  A copy
of the queue with one lock removed shows that the thread-sanitizer build catches a race."""
from __future__ import annotations

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HQ = os.path.join(ROOT, "tests", "host_queue")
QUEUE = os.path.join(ROOT, "paper_2402_15322_amd", "csrc", "queue.cpp")
SRCS = [os.path.join(HQ, "mock_solver.cpp"), os.path.join(HQ, "queue_check.cpp")]

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")


def _build_and_run(tmp_path, sanitize, queue_src=QUEUE):
    exe = tmp_path / f"qcheck_{sanitize.replace(',', '_')}"
    cmd = ["g++", "-std=c++17", "-O1", "-g", f"-fsanitize={sanitize}", "-fno-omit-frame-pointer",
           "-I", HQ, "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2402_15322_amd", "csrc"),
           queue_src] + SRCS + ["-o", str(exe), "-lpthread"]
    subprocess.check_call(cmd)
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=0 second_deadlock_stack=1",
               ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    return subprocess.run([str(exe)], capture_output=True, text=True, timeout=120, env=env)


def test_queue_host_logic_asan_ubsan(tmp_path):
    r = _build_and_run(tmp_path, "address,undefined")
    assert r.returncode == 0, r.stderr[-3000:]
    assert "queue host checks passed" in r.stdout
    assert "runtime error" not in r.stderr


def test_queue_host_logic_tsan(tmp_path):
    r = _build_and_run(tmp_path, "thread")
    assert r.returncode == 0, r.stderr[-3000:]
    assert "ThreadSanitizer" not in r.stderr
    assert "queue host checks passed" in r.stdout


def test_tsan_build_catches_a_planted_race(tmp_path):
    src = open(QUEUE).read()
    old = ("int se2_solve_queue_poll(se2_queue_t Q, uint64_t ticket, se2_report_t *report) {\n"
           "    if (!Q) return SE2_EINVAL;\n"
           "    std::lock_guard<std::mutex> lk(Q->mu);")
    assert old in src
    planted = tmp_path / "queue_race.cpp"
    planted.write_text(src.replace(old, old.rsplit("\n", 1)[0], 1))
    r = _build_and_run(tmp_path, "thread", str(planted))
    assert "data race" in r.stderr
