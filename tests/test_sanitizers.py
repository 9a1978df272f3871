"""Host sanitizer runs (AddressSanitizer with leak checks, and
UndefinedBehaviorSanitizer) of the FP64 oracle and of the C ABI's host code.
Each driver builds once per source change (tests/sanitize/build.py) and must
finish with no sanitizer report."""
import os
import subprocess

import pytest

from tests.sanitize import build as sanitize_build

ENV = dict(os.environ,
           ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
           OMP_NUM_THREADS="2")


def _run(exe: str, expect: str) -> None:
    r = subprocess.run([exe], env=ENV, capture_output=True, text=True, timeout=300)
    report = (r.stdout + r.stderr)[-6000:]
    assert r.returncode == 0, f"{os.path.basename(exe)} exited {r.returncode}\n{report}"
    assert "runtime error" not in r.stderr, report
    assert "ERROR: AddressSanitizer" not in r.stderr, report
    assert expect in r.stdout, report


def test_oracle_under_asan_and_ubsan():
    _run(sanitize_build.build_oracle(), "oracle sanitizer run: ok")


@pytest.mark.timeout(900)
def test_c_abi_host_code_under_asan_and_ubsan():
    _run(sanitize_build.build_capi(), "C ABI sanitizer run: ok")
