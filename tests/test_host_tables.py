"""The library's host-side table builder (csrc/tables.cpp: Gauss rules, basis
tables, the CFL spectral constant) built on the CPU with AddressSanitizer and
UndefinedBehaviorSanitizer, and checked against closed forms and the printed
spectral constants (tests/host_tables_check.cpp)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1403_1157_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_tables_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    exe = tmp_path / "host_tables_check"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-I", CSRC, os.path.join(CSRC, "tables.cpp"),
           os.path.join(ROOT, "tests", "host_tables_check.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0 and r.stdout.strip().endswith("OK"), r.stdout + r.stderr
