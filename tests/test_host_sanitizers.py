"""Host code checked on the CPU under the address and undefined-behaviour
sanitizers: the library's schedule of tet tiles with upwind cycles
(csrc/tet_schedule.cpp, plain C++) against brute force on random tiles with
planted cycles (tests/host/tet_schedule_check.cpp), and the oracle's C code
(oracle/sweep.c, oracle/cpu_sweep.c) on random block systems with cycles and
across thread counts (tests/host/oracle_c_check.c)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1910_11463_amd", "csrc")
ORACLE = os.path.join(ROOT, "oracle")
SAN_ENV = dict(os.environ, ASAN_OPTIONS="halt_on_error=1:detect_leaks=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _run(exe):
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=SAN_ENV)
    print(r.stdout, r.stderr)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("ok")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_tet_cycle_schedule_under_sanitizers(tmp_path):
    exe = str(tmp_path / "tet_schedule_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
           "-pthread", "-I" + CSRC, os.path.join(HERE, "host", "tet_schedule_check.cpp"),
           os.path.join(CSRC, "tet_schedule.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    _run(exe)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_c_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_c_check")
    cmd = ["gcc", "-std=c99", "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
           "-fopenmp", "-D_DEFAULT_SOURCE", os.path.join(HERE, "host", "oracle_c_check.c"),
           os.path.join(ORACLE, "sweep.c"), os.path.join(ORACLE, "cpu_sweep.c"), "-o", exe, "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    _run(exe)
