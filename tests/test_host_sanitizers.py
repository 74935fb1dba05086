"""The library's host-only dense routines (GMRES-polynomial least squares,
Hessenberg eigenvalues, Newton roots with added roots and Leja order,
numerical rank) under AddressSanitizer and UBSan.

The build makes a second host library of the same sources with
-fsanitize=address,undefined; the CPU tests of those routines run again in a
child process with the ASan runtime preloaded and that library selected, and
must pass with no sanitizer report."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN_LIB = os.path.join(ROOT, "paper_2508_17517_amd", "libairg_dense_host_san.so")


def _asan_runtime():
    try:
        out = subprocess.run(["g++", "-print-file-name=libasan.so"], capture_output=True, text=True,
                             timeout=60).stdout.strip()
    except (OSError, subprocess.SubprocessError):
        return None
    return out if out and os.path.isabs(out) and os.path.exists(out) else None


def test_dense_routines_pass_their_tests_under_asan_and_ubsan():
    assert os.path.exists(SAN_LIB), f"{SAN_LIB} is missing: run the build"
    # the library really is instrumented: it calls the sanitizers' runtimes
    syms = subprocess.run(["nm", "-D", SAN_LIB], capture_output=True, text=True, timeout=60).stdout
    assert "__asan_report_load8" in syms and "__ubsan_handle_" in syms
    rt = _asan_runtime()
    if rt is None:
        pytest.skip("no ASan runtime next to g++")
    env = dict(os.environ, LD_PRELOAD=rt, AIRG_HOST_LIB=SAN_LIB,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi.py"), "-k", "library"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    report = r.stdout[-3000:] + r.stderr[-3000:]
    assert r.returncode == 0, report
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, report
    assert " passed" in r.stdout and "failed" not in r.stdout, report
