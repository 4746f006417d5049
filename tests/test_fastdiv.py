"""The kernels' division by a fixed divisor (csrc/wd_fastdiv.h), compiled for
the host and checked against exact integer division: every divisor up to 4096
and large and power-of-two ones, at the dividends where a wrong multiplier or
shift would show first (multiples of d and their neighbours up to the 2^30
bound that every site and block index stays below) and at random ones."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_fastdiv_matches_integer_division(tmp_path):
    exe = str(tmp_path / "fastdiv_check")
    subprocess.run(["g++", "-O2", "-std=c++17", "-Wall", "-Werror",
                    "-I", os.path.join(ROOT, "paper_2409_03030_amd", "csrc"),
                    os.path.join(ROOT, "tests", "fastdiv_check.cpp"), "-o", exe], check=True)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.startswith("ok "), out.stdout
    assert int(out.stdout.split()[1]) > 10**8
