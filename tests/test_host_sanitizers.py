"""CPU: the library's host code and the oracle under sanitizers. The
planner's scheduler (against fake executors) and the host functions build
with g++ under AddressSanitizer + UndefinedBehaviorSanitizer and under
ThreadSanitizer (tests/host/host_checks.cpp); the oracle builds with gcc
under AddressSanitizer + UndefinedBehaviorSanitizer (tests/host/
oracle_checks.c). Each program must run clean: any sanitizer report makes
it exit non-zero."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HOST = os.path.join(HERE, "host")
CSRC = os.path.join(ROOT, "paper_2509_16079_amd", "csrc")
BUILD = os.path.join(HOST, "_build")
HOST_SOURCES = [os.path.join(CSRC, f) for f in ("host.cpp", "sampling.cpp", "plate_system.cpp")]
SAN_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=23",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=24",
               TSAN_OPTIONS="halt_on_error=1:exitcode=25", OMP_NUM_THREADS="1")

pytestmark = pytest.mark.skipif(shutil.which("g++") is None or shutil.which("gcc") is None,
                                reason="needs gcc and g++")


def _build_and_run(cmd, exe, timeout=300):
    os.makedirs(BUILD, exist_ok=True)
    b = subprocess.run(cmd + ["-o", exe], capture_output=True, text=True, timeout=600)
    assert b.returncode == 0, b.stderr[-4000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=timeout, env=SAN_ENV)
    assert r.returncode == 0, (r.returncode, r.stdout[-2000:], r.stderr[-6000:])
    assert "ALL OK" in r.stdout
    assert "Sanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-6000:]
    return r.stdout


CXX = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-I",
       os.path.join(ROOT, "include"), "-I", CSRC, os.path.join(HOST, "host_checks.cpp")] + \
    HOST_SOURCES


def test_host_code_under_address_and_undefined_sanitizers():
    out = _build_and_run(CXX + ["-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                                "-pthread"], os.path.join(BUILD, "host_asan"))
    for name in ("host_functions", "serial_and_concurrent", "budget", "ticket_life_cycle",
                 "latency_bookkeeping", "failing_executor", "concurrent_clients"):
        assert "ok " + name in out


# ThreadSanitizer needs a runtime that intercepts pthread_cond_clockwait
# (std::condition_variable::wait_for on a steady clock); GCC 11's does not and
# reports false double locks, so this build takes the image's LLVM clang++.
CLANGXX = "/opt/rocm/llvm/bin/clang++"


@pytest.mark.skipif(not os.path.exists(CLANGXX), reason="needs the ROCm LLVM clang++")
def test_planner_scheduler_under_thread_sanitizer():
    _build_and_run([CLANGXX] + CXX[1:] + ["-fsanitize=thread", "-pthread"],
                   os.path.join(BUILD, "host_tsan"))


def test_oracle_under_address_and_undefined_sanitizers():
    cmd = ["gcc", "-std=c11", "-D_DEFAULT_SOURCE", "-O1", "-g", "-fno-omit-frame-pointer",
           "-ffp-contract=off", "-fopenmp", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-I", os.path.join(ROOT, "oracle"),
           os.path.join(ROOT, "oracle", "vpm_oracle.c"), os.path.join(HOST, "oracle_checks.c"),
           "-lm"]
    _build_and_run(cmd, os.path.join(BUILD, "oracle_asan"))
