"""The library's device-free planning code (csrc/host_plan.h: the sector
kernel's LDS layout, the factorization of each group's sector-form
coefficients of Section 2.4, the batched launch's work list) built with the
host compiler under AddressSanitizer and UndefinedBehaviorSanitizer, and
its checks run (tests/host/host_plan_check.cpp).  No GPU is involved."""

import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_host_plan_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "host_plan_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-Wall", "-Wextra", "-Werror",
           os.path.join(HERE, "host", "host_plan_check.cpp"), "-o", exe]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    assert run.returncode == 0, run.stdout + run.stderr
    assert "all host plan checks passed" in run.stdout
    assert "runtime error" not in run.stderr and "AddressSanitizer" not in run.stderr
