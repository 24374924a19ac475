"""The host code of libcomposite.so under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU only).

The library's sources are rebuilt with the host pass instrumented, and the
CPU suites that drive its host code without a GPU (argument checks of every
entry point, status strings, the banded-compositing orchestration with its
error paths, the ABI layout checks) run against that build in a child
process with the clang ASan runtime preloaded.  Any sanitizer report fails
the test."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SUITES = ["tests/test_abi_cpu.py", "tests/test_subdivide_cpu.py", "tests/test_fingerprint_cpu.py"]


@pytest.mark.timeout(600)
def test_host_code_clean_under_asan_and_ubsan():
    if os.environ.get("LD_PRELOAD") or os.path.exists("/etc/ld.so.preload"):
        pytest.skip("a preload is already configured here; the ASan runtime must load first")
    from paper_2104_14667_amd import build
    if not os.path.exists(build.HIPCC):
        pytest.skip("hipcc not available")
    lib = build.build_host_sanitized()
    env = dict(os.environ,
               LD_PRELOAD=build.sanitizer_runtime(),
               COMPOSITE_LIBRARY=lib,
               # the interpreter itself is not instrumented and keeps its
               # allocations to the end: leak reports would be its, not ours
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1",
               HIP_VISIBLE_DEVICES=os.environ.get("HIP_VISIBLE_DEVICES", ""))
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        "-m", "not gpu", *SUITES],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=540)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out, out[-4000:]
    assert "runtime error:" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert " passed" in r.stdout
