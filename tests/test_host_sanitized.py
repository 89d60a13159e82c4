"""The host C++ of the library (C-ABI entry points, argument checks, plan and
list construction, tables, stencil) under AddressSanitizer and
UndefinedBehaviorSanitizer, on the CPU.

The sanitized copy of the library is built beside the regular one (host
sources compiled by clang with -fsanitize=address,undefined, device objects
shared with the regular build) and the host-logic tests run against it in a
child process with the sanitizer runtime preloaded.  Any report (a heap or
stack overflow, a use after free, undefined behaviour) ends that process
with an error, so the test fails with the report in its output.  Leak
checking is off: the Python interpreter itself keeps allocations alive at
exit."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_host_code_is_clean_under_asan_and_ubsan():
    from paper_2211_14537_amd import build as B
    try:
        runtime = B.sanitizer_runtime()
    except RuntimeError as e:
        pytest.skip(str(e))
    lib = B.build_host_sanitized()
    env = dict(os.environ)
    env.update({
        "LD_PRELOAD": runtime,
        "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0:exitcode=86",
        "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1:exitcode=87",
        "VFX_LIBRARY": lib,
    })
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider",
           os.path.join(ROOT, "tests", "test_library_host.py")]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=1200)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-6000:]
    assert r.returncode == 0, out[-6000:]
    assert " passed" in out
