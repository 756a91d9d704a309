"""The host planner under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only): planner.cpp and a driver (tests/asan/planner_fuzz.cpp) built with
g++, then random gate streams over every gate kind, 1-32 qubits and bound
parameters go through normalisation, planning with four option sets
(windows off / 4 / 5 / 6, fixed and per-group tile geometry, random tile
sizes), description, inversion, gradient bookkeeping, GF(2) kernel arguments
and numeric tables.  Any sanitizer report fails the test."""
import os
import re
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2609_19147_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_planner_fuzz_under_asan_ubsan():
    flags = ["-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
             "-I", os.path.join(ROOT, "include"), "-I", CSRC]
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "planner_fuzz")
        r = subprocess.run(["g++", *flags, os.path.join(HERE, "asan", "planner_fuzz.cpp"),
                            os.path.join(CSRC, "planner.cpp"), "-o", exe], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-4000:]
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
        r = subprocess.run([exe, "150"], capture_output=True, text=True, env=env, timeout=600)
        assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
        assert "plans ok: 600" in r.stdout and "runtime error" not in r.stderr, r.stdout + r.stderr[-2000:]
        # the neighbour masks of pair-mismatch diagonal groups were checked
        # against direct counts on some of the random streams
        m = re.search(r"pair-neighbour checks: (\d+)", r.stdout)
        assert m and int(m.group(1)) > 0, r.stdout
