"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer.

The C ABI's host side (argument validation, workspace layout, material
tables, the scheduler's bookkeeping) is compiled with both sanitizers on its
host pass (``build.build_host_sanitized``; device code unchanged) and the
CPU tests of the ABI run against that build in a child process with the
sanitizer runtime preloaded.  Any report (out-of-bounds access, use after
free, undefined behaviour) fails the child and this test.  Needs the device
units of a previous build() and hipcc; skipped otherwise.
"""
import os
import shutil
import subprocess
import sys

import pytest

from paper_1411_0330_amd import build as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _ready():
    if shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"):
        return "hipcc not found"
    for src, obj, _ in B.UNITS:
        if src != "runtime.hip" and not os.path.exists(os.path.join(B.OBJDIR, obj)):
            return "device units not built"
    if not os.path.exists(B.sanitizer_runtime()):
        return "sanitizer runtime not found"
    return None


@pytest.mark.timeout(600)
def test_abi_host_code_is_clean_under_asan_and_ubsan():
    why = _ready()
    if why:
        pytest.skip(why)
    lib = B.build_host_sanitized()
    env = dict(os.environ)
    env.update({
        "LD_PRELOAD": B.sanitizer_runtime(),
        "ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:abort_on_error=0",
        "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
        "LSH_LIB_PATH": lib,
    })
    proc = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider",
                           os.path.join(ROOT, "tests", "test_abi.py")],
                          cwd=ROOT, env=env, capture_output=True, text=True, timeout=540)
    out = proc.stdout + proc.stderr
    assert proc.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert " passed" in out
