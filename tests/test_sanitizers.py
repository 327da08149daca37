"""The host code (network checks, host absorption, planner, search, slicer,
analysis) under AddressSanitizer and UndefinedBehaviorSanitizer, on the CPU.

The library is rebuilt with the sanitizers bound to the host compiler and
loaded in a fresh interpreter with the sanitizer runtime preloaded; the host
tests then run against it.  Any invalid access or undefined behaviour aborts
that interpreter with a report, which fails this test.  No kernel runs here.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.slow
def test_host_tests_pass_under_asan_and_ubsan():
    sys.path.insert(0, ROOT)
    from paper_2407_00769_amd import build as b
    try:
        lib = b.build_sanitized()
    except RuntimeError as e:   # a missing toolchain is not a finding
        pytest.skip(f"sanitizer build unavailable: {e}")
    rt = b.sanitizer_runtime()
    if not os.path.exists(rt):
        pytest.skip("clang AddressSanitizer runtime not found")
    env = dict(os.environ)
    env.update(TNC_LIB=lib, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
                        os.path.join(ROOT, "tests", "test_host.py"), os.path.join(ROOT, "tests", "test_bench_host.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    tail = (r.stdout + r.stderr)[-6000:]
    assert r.returncode == 0, tail
    assert "passed" in r.stdout, tail
