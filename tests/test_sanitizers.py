"""Sanitizer builds of the CPU-side code, run on the host (no GPU).

* the oracle (every entry point, threaded drivers included) under
  AddressSanitizer + UndefinedBehaviorSanitizer, and its threaded drivers
  under ThreadSanitizer, through tests/sanitize/oracle_driver.c;
* the library's host code (input validation, class tables, the 128-bit null
  count) and the seeded input generators under AddressSanitizer +
  UndefinedBehaviorSanitizer, through tests/sanitize/host_driver.cpp.

Each driver exits non-zero on a disagreement; a sanitizer report aborts it.
GPU code is not built here: the device kernels are covered by the parity
tests on the GPU."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = [os.path.join(ROOT, "oracle", f) for f in
          ("census_oracle.c", "brute.c", "wedge.c", "selftest.c", "labelled.c")]
SAN = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_1209_6308_amd", "csrc")
ENV = dict(os.environ,
           ASAN_OPTIONS="halt_on_error=1:abort_on_error=0:detect_leaks=1",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
           TSAN_OPTIONS="halt_on_error=1:second_deadlock_stack=1")


def _build(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "cannot find" in r.stderr and "san" in r.stderr:
        pytest.skip("sanitizer runtime not installed: " + r.stderr.strip().splitlines()[-1])
    assert r.returncode == 0, r.stderr


def _run(exe):
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "Sanitizer" not in r.stderr, r.stderr
    return r.stdout


def test_oracle_address_and_undefined(tmp_path):
    exe = str(tmp_path / "oracle_asan")
    _build(["gcc", "-O1", "-g", "-std=gnu11", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
            "-fno-omit-frame-pointer", *ORACLE, os.path.join(SAN, "oracle_driver.c"), "-o", exe, "-lpthread"])
    assert "0 disagreement" in _run(exe)


def test_oracle_threads(tmp_path):
    exe = str(tmp_path / "oracle_tsan")
    _build(["gcc", "-O1", "-g", "-std=gnu11", "-fsanitize=thread", *ORACLE, os.path.join(SAN, "oracle_driver.c"),
            "-o", exe, "-lpthread"])
    assert "0 disagreement" in _run(exe)


def test_host_code_address_and_undefined(tmp_path):
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    exe = str(tmp_path / "host_asan")
    _build(["g++", "-O1", "-g", "-std=c++17", "-fopenmp", "-fsanitize=address,undefined",
            "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-D__HIP_PLATFORM_AMD__",
            "-I" + os.path.join(rocm, "include"), "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
            os.path.join(CSRC, "host.cpp"), os.path.join(ROOT, "paper_1209_6308_amd", "gen", "graphgen.cpp"),
            os.path.join(SAN, "host_driver.cpp"), "-o", exe, "-L" + os.path.join(rocm, "lib"), "-lamdhip64",
            "-Wl,-rpath," + os.path.join(rocm, "lib")])
    assert "0 failed" in _run(exe)
