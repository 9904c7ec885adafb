"""AddressSanitizer and UndefinedBehaviorSanitizer runs of host code (CPU).

* the oracle (oracle/okpz_oracle.c) with the driver tests/c/oracle_check.c;
* the library's host-only logic (paper_1110_6745_amd/csrc/host_logic.cpp:
  slope-field and checkpoint validation, measurement times) with the driver
  tests/c/host_logic_check.cpp.

Both are compiled with gcc/g++ only (no device code) and must run clean:
any sanitizer report aborts the program.
"""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", OMP_NUM_THREADS="2",
           UBSAN_OPTIONS="print_stacktrace=1")


def _run(exe, expect):
    out = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=ENV)
    assert out.returncode == 0, out.stderr[-4000:]
    assert out.stdout.strip() == expect
    assert "runtime error" not in out.stderr


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_check")
    subprocess.run(["gcc", "-std=gnu11", "-fopenmp", *SAN,
                    os.path.join(ROOT, "oracle", "okpz_oracle.c"),
                    os.path.join(ROOT, "tests", "c", "oracle_check.c"), "-o", exe, "-lm"],
                   check=True)
    _run(exe, "oracle ok")


def test_host_logic_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_logic_check")
    csrc = os.path.join(ROOT, "paper_1110_6745_amd", "csrc")
    subprocess.run(["g++", "-std=c++17", "-Wall", "-Wextra", *SAN, "-I", csrc,
                    os.path.join(csrc, "host_logic.cpp"),
                    os.path.join(ROOT, "tests", "c", "host_logic_check.cpp"), "-o", exe],
                   check=True)
    _run(exe, "host logic ok")
