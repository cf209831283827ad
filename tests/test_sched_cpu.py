"""The serving scheduler (csrc/tsa_sched.hpp) on the CPU, driving a fake
executor with controllable batch and scan times (tests/sched/fake_sched.cpp):
FIFO order per class, batches by cube, admission by slots and by scratch
budget, shared full-cube scans, drain timeouts, launch failures, replay and
many submitting threads -- built plainly and under ThreadSanitizer."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "sched", "fake_sched.cpp")
# GCC 11's ThreadSanitizer runtime in this image reports races between two
# holders of one mutex; the LLVM runtime of the ROCm toolchain does not (and
# does report a planted race), so the sanitizer build uses it.
CLANG = "/opt/rocm/llvm/bin/clang++"


def _run(tmp_path, cxx, flags, env=None):
    exe = os.path.join(str(tmp_path), "fake_sched")
    cmd = [cxx, "-std=c++17", "-g", "-pthread", *flags, SRC, "-o", exe]
    b = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert b.returncode == 0, b.stderr[-4000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env={**os.environ, **(env or {})})
    return r.returncode, r.stdout + r.stderr


def test_scheduler_with_fake_executor(tmp_path):
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    rc, out = _run(tmp_path, cxx, ["-O2", "-Wall", "-Wextra", "-Werror"])
    assert rc == 0 and "all ok" in out, out[-4000:]


def test_scheduler_under_thread_sanitizer(tmp_path):
    if not os.path.exists(CLANG):
        pytest.skip("no LLVM ThreadSanitizer toolchain")
    rc, out = _run(tmp_path, CLANG, ["-O1", "-fsanitize=thread"],
                   env={"TSAN_OPTIONS": "halt_on_error=1 exitcode=66"})
    assert "ThreadSanitizer" not in out, out[-6000:]
    assert rc == 0 and "all ok" in out, out[-4000:]
