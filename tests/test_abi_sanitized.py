"""The C ABI's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

A copy of the library whose host code (argument and descriptor checks,
FFT factorisation, planning) is built with -fsanitize=address,undefined
runs the CPU-side ABI and binding tests in a child process with the clang
ASan runtime preloaded; any sanitizer report aborts that child and fails
this test.  Device code is built as usual and never runs here."""
import os
import subprocess
import sys

import pytest

from paper_0912_4255_amd import build as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _stale():
    if not os.path.exists(B.SAN_LIB):
        return True
    t = os.path.getmtime(B.SAN_LIB)
    deps = [os.path.join(B.CSRC, f) for f in os.listdir(B.CSRC)] + [os.path.join(ROOT, "include", "rsfstat.h")]
    return any(os.path.getmtime(d) > t for d in deps)


def test_abi_host_paths_clean_under_asan_ubsan():
    rt = B.san_runtime()
    if rt is None:
        pytest.skip("clang ASan runtime not found")
    if _stale():
        B.build(sanitize=True)
    env = dict(os.environ)
    env.update(LD_PRELOAD=rt, RSF_LIB=B.SAN_LIB,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
           os.path.join(ROOT, "tests", "test_abi_cpu.py"), os.path.join(ROOT, "tests", "test_binding_shapes_cpu.py")]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert " passed" in out
