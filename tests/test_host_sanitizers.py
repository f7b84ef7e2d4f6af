"""The library's plain C++ host code (plan, symbolic factorization, dense
small eigensolver, Krylov-Schur cycle, worker pool) built with g++ under the
address + undefined-behaviour sanitizers and under the thread sanitizer, and
run through tests/host/sanitize_main.cpp.  CPU only; no HIP source is built."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2112_14064_amd", "csrc")
MAIN = os.path.join(ROOT, "tests", "host", "sanitize_main.cpp")
HOST_SOURCES = ["plan.cpp", "small_eig.cpp", "ks_host.cpp"]

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")


def _build_and_run(tmp_path, flags, mode):
    exe = str(tmp_path / f"host_{mode}")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", *flags, "-I", CSRC, MAIN,
           *[os.path.join(CSRC, s) for s in HOST_SOURCES], "-o", exe, "-pthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    # the environment is passed on unchanged; a library preloaded by the
    # environment may precede the sanitizer runtime, which is allowed here
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", TSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([exe, mode], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-6000:])
    assert "host checks ok" in r.stdout


def test_host_code_under_address_and_ub_sanitizers(tmp_path):
    _build_and_run(tmp_path, ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"], "asan")


def test_worker_pool_under_thread_sanitizer(tmp_path):
    _build_and_run(tmp_path, ["-fsanitize=thread"], "tsan")
