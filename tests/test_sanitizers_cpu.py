"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU).

The host side of libbtdf (argument checks, layout, marker binning, the
calibration's dense solve) is rebuilt with both sanitizers in its host
pass, and the CPU tests of the C ABI run against that build; the FP64
oracle is rebuilt the same way with gcc and its pins run against it. Each
run is a child process with the sanitizer runtime preloaded, so a report
(heap overflow, use after free, signed overflow, misaligned access ...)
fails the run. Leak checks are off: the Python interpreter itself keeps
allocations alive until exit.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
           "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"}
ORACLE_PINS = ["tests/test_oracle_delta.py", "tests/test_oracle_lbm.py", "tests/test_oracle_ib.py",
               "tests/test_oracle_bc.py", "tests/test_oracle_inlet.py", "tests/test_oracle_moving.py"]


def run_tests(files, env):
    full = dict(os.environ)
    full.update(SAN_ENV)
    full.update(env)
    full["OMP_NUM_THREADS"] = "2"
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu"] + files
    r = subprocess.run(cmd, cwd=ROOT, env=full, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-4000:]
    assert "passed" in r.stdout


@pytest.mark.slow
def test_abi_host_code_under_sanitizers():
    from paper_1806_09403_amd import build
    lib = build.build(sanitize=True)
    run_tests(["tests/test_abi_cpu.py"], {"BTDF_LIBRARY": lib, "LD_PRELOAD": build.san_runtime()})


@pytest.mark.slow
def test_oracle_pins_under_sanitizers():
    from oracle import build
    lib = build.build(sanitize=True)
    run_tests(ORACLE_PINS, {"ORACLE_LIBRARY": lib, "LD_PRELOAD": build.san_runtime()})
