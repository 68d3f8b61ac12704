"""The host code under the address and undefined-behaviour sanitizers (CPU only).

mech.cpp and api.cpp are built by the host compiler with the sanitizers into a host-only
library (launchers that report a missing device), and the host ABI tests run against it
in a child process that preloads the sanitizer runtime: mechanism loading with device -1,
malformed, truncated, corrupted and unbalanced files, and the argument validation of every
entry point.  Any sanitizer report aborts the child and fails this test.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def sanitized(tmp_path_factory):
    from paper_2409_06404_amd.build import build_host_only_library, host_sanitizer_runtime
    if shutil.which("g++") is None:
        pytest.skip("no host C++ compiler")
    rt = host_sanitizer_runtime()
    if rt is None:
        pytest.skip("no address-sanitizer runtime")
    out = str(tmp_path_factory.mktemp("san") / "libcrf_san.so")
    build_host_only_library(out, sanitize=True)
    env = dict(os.environ, CRF_LIB=out, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    return out, env


def test_library_is_instrumented(sanitized):
    out, _ = sanitized
    syms = subprocess.run(["nm", "-D", out], capture_output=True, text=True).stdout
    assert "__asan_report_load8" in syms and "__ubsan_handle_" in syms


def test_host_abi_tests_under_sanitizers(sanitized):
    out, env = sanitized
    probe = subprocess.run([sys.executable, "-c", "from paper_2409_06404_amd import _lib; _lib.lib(); "
                            "print(_lib.LIB_PATH)"], cwd=ROOT, env=env, capture_output=True, text=True)
    assert probe.returncode == 0 and probe.stdout.strip() == out, probe.stderr[-2000:]
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                        os.path.join("tests", "test_abi_host.py")], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=900)
    tail = (r.stdout + r.stderr)[-4000:]
    assert r.returncode == 0, tail
    assert "AddressSanitizer" not in tail and "runtime error" not in tail, tail
    assert " passed" in tail
