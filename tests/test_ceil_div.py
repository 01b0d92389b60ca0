"""The propagation kernel's ceiling division (csrc/propagate.hip:
ceil_div_small): the truncated float quotient with the reciprocal one ulp
either side of 1/q, corrected by one integer product, equals ceil(r / q)
for every 0 < q < r up to the diagonal of a 20 km cell and on a sample up
to 2^16 - 1 (metres left on an axis are below 2^16).  The correction is
needed on many pairs, so dropping it fails."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_ceil_div_small_is_exact(tmp_path):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    exe = tmp_path / "ceil_div_check"
    subprocess.run([cc, "-std=c11", "-O2", "-ffp-contract=off", os.path.join(ROOT, "tests", "ceil_div_check.c"),
                    "-o", str(exe), "-lm"], check=True)
    n, bad, corrected = map(int, subprocess.run([str(exe)], check=True, capture_output=True,
                                                 text=True).stdout.split())
    assert n > 400_000_000
    assert bad == 0
    assert corrected > 1_000_000
