"""The library's host code under AddressSanitizer and
UndefinedBehaviorSanitizer: geometry, trimmed layout, ring lengths, launch
plans, the chunked decode's transfer matrices (threaded symbolic sweep) and
the plans' host checks, run from a process with the sanitizer runtime
preloaded.  Needs the sanitized build (python -m paper_1504_07038_amd.build
--sanitize, a few minutes); skipped when it is absent."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_host_code_is_clean_under_sanitizers():
    from paper_1504_07038_amd import build

    if not os.path.exists(build.SAN_LIB):
        pytest.skip("sanitized library not built (python -m paper_1504_07038_amd.build --sanitize)")
    rt = build.sanitizer_runtime()
    assert rt, "AddressSanitizer runtime not found"
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    res = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "san_driver.py"),
                          build.SAN_LIB], env=env, capture_output=True, text=True, timeout=600)
    assert res.returncode == 0, res.stdout[-2000:] + res.stderr[-4000:]
    assert "AddressSanitizer" not in res.stderr and "runtime error" not in res.stderr
    assert "checks passed" in res.stdout
