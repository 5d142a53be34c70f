"""The CPU suite once more, against builds of the library's host code and of the C oracle
made with AddressSanitizer and UndefinedBehaviorSanitizer, in a child interpreter with
clang's ASan runtime preloaded.  An out-of-bounds access, a use after free or undefined
behaviour in the plan, layout, tiling, autotuner-cache, ranker-host, plain-path or
plan-generator code, or in the oracle's C, ends the child with a report.  (The kernel
sources keep their ordinary objects: only host code is instrumented, and nothing here
launches a kernel.)"""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
# the one slow oracle test (a 64-seed Monte Carlo, minutes without OpenMP under ASan)
SLOW = "tests/test_oracle_search.py::test_injected_pulse_recovered_at_analytic_snr"


def _asan_runtime():
    found = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return found[-1] if found else None


def test_cpu_suite_under_host_sanitizers(tmp_path):
    rt = _asan_runtime()
    if rt is None or not os.path.exists("/opt/rocm/bin/hipcc"):
        pytest.skip("clang's ASan runtime or hipcc is not installed")
    from paper_2606_27262_amd import build as B
    import oracle
    lib = B.build_host_sanitized(str(tmp_path / "lib"))
    olib = oracle.build_sanitized(str(tmp_path / "liboracle_san.so"))
    env = dict(os.environ, LD_PRELOAD=rt, SPL_LIBRARY=lib, SPL_ORACLE_LIBRARY=olib,
               ASAN_OPTIONS="detect_leaks=0:detect_odr_violation=0:alloc_dealloc_mismatch=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    # -s: a report printed just before the child aborts must reach this pipe
    cmd = [sys.executable, "-m", "pytest", "tests", "-q", "-s", "-m", "not gpu", "-p", "no:cacheprovider",
           "--ignore", os.path.relpath(os.path.abspath(__file__), ROOT), "--deselect", SLOW]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=1200)
    out = r.stdout + r.stderr
    tail = out[-4000:]
    assert "runtime error:" not in out, tail
    assert "ERROR: AddressSanitizer" not in out, tail
    assert r.returncode == 0, tail
    assert " passed" in out, tail
