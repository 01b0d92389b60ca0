"""The FP64 logarithm of the rate path (csrc/ln64.h), built for the host and
compared with the C library's log over the normal range, near 1, across the
[sqrt(1/2), sqrt(2)) split, on (0, 1) and at special values."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_ln_f64_within_one_ulp_of_libm(tmp_path):
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    exe = tmp_path / "ln64_check"
    subprocess.run([cxx, "-std=c++17", "-O2", "-ffp-contract=off", "-D__host__=", "-D__device__=",
                    "-I", os.path.join(ROOT, "paper_1905_09317_amd", "csrc"),
                    os.path.join(ROOT, "tests", "ln64_check.cpp"), "-o", str(exe)], check=True)
    n, worst, worst_x, bad_special = subprocess.run([str(exe)], check=True, capture_output=True,
                                                    text=True).stdout.split()
    assert int(n) >= 2_000_000
    assert int(bad_special) == 0
    assert float(worst) <= 1.0, f"{worst} ulp at {worst_x}"
