"""The C-ABI's CPU checks (tests/test_abi.py) rerun against a build whose host
code carries AddressSanitizer and UndefinedBehaviorSanitizer (every argument
check, plan validation and status path of the library's host side), with no
device visible.  Any out-of-bounds access, use after free or undefined
behaviour on those paths aborts the run."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_abi_checks_under_host_sanitizers():
    from paper_2209_15040_amd import build
    rt = build.asan_runtime()
    if not rt:
        pytest.skip("no ASan runtime in this ROCm")
    lib = build.build_host_sanitized()
    if not lib:
        pytest.skip("kernel objects of a regular build are missing (python -m paper_2209_15040_amd.build)")
    env = dict(os.environ, LD_PRELOAD=rt, WSFFT_ABI_LIB=lib, WSFFT_ABI_NO_TORCH="1", HIP_VISIBLE_DEVICES="",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_abi.py"), "-q",
                        "-p", "no:cacheprovider", "-x"], env=env, capture_output=True, text=True, timeout=600,
                       cwd=ROOT)
    print(r.stdout[-3000:], r.stderr[-3000:])
    assert r.returncode == 0
    assert "passed" in r.stdout
