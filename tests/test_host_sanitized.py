"""CPU test: the library's host code built with AddressSanitizer and UndefinedBehaviorSanitizer
(device code unchanged) and driven by tests/host_asan_check.cpp: argument validation of the C
ABI, the host argument checks, the quadrature and the short-range polynomial table.  Any
memory error or undefined behaviour aborts the driver."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.timeout(900)
def test_host_code_under_sanitizers():
    from paper_2510_26611_amd import build_lib
    exe = build_lib.build_host_sanitized(os.path.join(HERE, "host_asan_check.cpp"))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "host checks passed" in r.stdout
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
