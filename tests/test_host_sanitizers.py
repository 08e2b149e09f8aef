"""The host planner built with AddressSanitizer and UndefinedBehaviorSanitizer (g++, host code
only) and driven over every pair of input and output orders for r <= 5, a sample for r = 6..8,
every schedule, with and without kept buckets (tests/host/plan_check.cpp).  CPU only."""
import os
import shutil
import subprocess
import tempfile

import pytest

from conftest import ROOT

CSRC = os.path.join(ROOT, "paper_2005_10427_amd", "csrc")
FLAGS = ["-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
         "-fno-omit-frame-pointer"]


def _gxx():
    gxx = shutil.which("g++")
    if not gxx:
        pytest.skip("g++ not available")
    return gxx


def test_planner_under_address_and_undefined_behaviour_sanitizers():
    gxx = _gxx()
    with tempfile.TemporaryDirectory(prefix="qsd_san_") as tmp:
        exe = os.path.join(tmp, "plan_check")
        build = subprocess.run([gxx] + FLAGS + ["-I" + CSRC, os.path.join(CSRC, "plan.cpp"),
                                                os.path.join(ROOT, "tests", "host", "plan_check.cpp"), "-o", exe],
                               capture_output=True, text=True)
        if build.returncode != 0 and "sanitize" in build.stderr and "cannot find" in build.stderr:
            pytest.skip("sanitizer runtimes not installed")
        assert build.returncode == 0, build.stderr
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
                   UBSAN_OPTIONS="print_stacktrace=1")
        run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
        assert run.returncode == 0, run.stdout[-2000:] + run.stderr[-4000:]
        assert run.stdout.strip().endswith("ok"), run.stdout[-2000:]
