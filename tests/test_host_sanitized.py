"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

libtg.so is rebuilt with both sanitizers in its host code (the AR-chain with
its thread pool and vector clones, the chain membership) and the CPU tests
of that code run against it in a subprocess with the sanitizer runtime
preloaded.  An out-of-bounds access, a use after free or an undefined
operation aborts the run and fails this test with the report.
"""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_host_code_under_address_and_undefined_sanitizers(tmp_path):
    rt = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not rt:
        pytest.skip("no clang ASan runtime")
    from paper_1507_01009_amd import build as B
    lib = B.build_host_sanitized(str(tmp_path / "libtg_san.so"))
    env = dict(os.environ)
    env.update({
        "TG_LIB": lib,
        "LD_PRELOAD": rt[-1],
        "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
        "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1",
        "PYTHONPATH": ROOT + os.pathsep + env.get("PYTHONPATH", ""),
    })
    tests = ["tests/test_archain.py", "tests/test_archain_threads.py", "tests/test_membership.py"]
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        *tests], cwd=ROOT, env=env, capture_output=True, text=True, timeout=1200)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-5000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-5000:]
