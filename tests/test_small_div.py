"""The ceiling division of the axis stepping (csrc/small_div.h), built for
the host and compared with integer division for every dividend up to the
longest axis (28285 m) and every divisor up to it, with reciprocals up to
two ulp off the correctly rounded value."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_ceil_div_small_exhaustive(tmp_path):
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    exe = tmp_path / "small_div_check"
    subprocess.run([cxx, "-std=c++17", "-O2", "-ffp-contract=off", "-D__host__=", "-D__device__=",
                    "-I", os.path.join(ROOT, "paper_1905_09317_amd", "csrc"),
                    os.path.join(ROOT, "tests", "small_div_check.cpp"), "-o", str(exe)], check=True)
    bad, n = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()[-2:]
    assert int(n) == 1_200_273_975
    assert int(bad) == 0
