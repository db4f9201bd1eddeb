"""The serving scheduler (csrc/sched.hpp, host-only C++) against a fake
executor, on the CPU: FIFO admission, a workspace budget that holds only a few
requests, rejection of a request that can never fit, failure isolation (a
batch that fails at launch or while running fails only its own requests),
latency from the stated arrival, and launches outside the scheduler's lock.
The cases live in tests/sched_mock.cpp, compiled here with g++."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "sched_mock.cpp")


def test_scheduler_with_fake_executor(tmp_path):
    exe = str(tmp_path / "sched_mock")
    cmd = ["g++", "-std=c++17", "-O1", "-pthread", "-Wall", "-Werror",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2606_09318_amd", "csrc"),
           SRC, "-o", exe]
    subprocess.run(cmd, check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    done = [ln.split()[1] for ln in r.stdout.splitlines() if ln.startswith("ok ")]
    assert done == ["fifo", "tiny_budget", "oversize_rejected_alone", "failure_isolation_launch",
                    "failure_isolation_running", "latency_from_arrival", "launch_outside_lock"]


def test_scheduler_under_thread_sanitizer(tmp_path):
    """The same cases built with ThreadSanitizer (host code only): the worker
    thread, submissions and polls share the scheduler's state without races."""
    exe = str(tmp_path / "sched_mock_tsan")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-pthread", "-fsanitize=thread",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2606_09318_amd", "csrc"),
           SRC, "-o", exe]
    if subprocess.run(cmd, capture_output=True).returncode != 0:
        import pytest
        pytest.skip("g++ cannot build with -fsanitize=thread here")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300,
                       env=dict(os.environ, TSAN_OPTIONS="halt_on_error=1"))
    assert r.returncode == 0, r.stdout + r.stderr[-4000:]
