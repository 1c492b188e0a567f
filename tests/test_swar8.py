"""The 8-bit-lane local recurrence that the int8 cell-rate probe issues
(csrc/swar8.h), checked on the CPU: byte maxima, the byte-permute sign
spread emulated from its selector definition, and a 16-row column for four
targets against the exact local recurrence, the guard bits against an exact
overflow test.  The probe's rate is only meaningful for a correct
recurrence."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_swar8_column(tmp_path):
    gxx = shutil.which("g++")
    if not gxx:
        pytest.skip("g++ not found")
    exe = str(tmp_path / "swar8_check")
    subprocess.run([gxx, "-O2", "-std=c++17", "-D__host__=", "-D__device__=", "-Wall", "-Werror",
                    "-Wno-unknown-pragmas", "-I", os.path.join(ROOT, "paper_1701_01575_amd", "csrc"),
                    os.path.join(ROOT, "tests", "swar8_check.cpp"), "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.startswith("ok"), r.stdout + r.stderr
