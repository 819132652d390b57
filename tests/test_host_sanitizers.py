"""The host-side C-ABI checks (tests/test_abi_host.py) run again against a copy
of libddx.so whose host code is built with AddressSanitizer and
UndefinedBehaviorSanitizer: argument validation, descriptor copies, call-order
state, blocking, the host tables of the Chirpolator, image, incoherent and
Chimageator entry points.  Any sanitizer report aborts the child run.  No GPU
is used (the checks touch none)."""
import os
import shutil
import subprocess
import sys

import pytest

from paper_1109_3186_amd import build as b

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which(os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")) is None, reason="hipcc not found")
def test_host_abi_checks_under_asan_and_ubsan():
    lib = b.build_sanitized()
    env = dict(os.environ)
    env.update({
        "DDX_LIB_PATH": lib,
        "LD_PRELOAD": b.sanitizer_runtime(),
        # Python itself is not instrumented: its allocations are not leaks of ours
        "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1:halt_on_error=1",
        "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1",
    })
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi_host.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-6000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out[-6000:]
    assert " passed" in out
