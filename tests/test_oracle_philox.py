"""Pins for the oracle's Philox4x32-10: published known answers and rocRAND."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat(golden_dir):
    rows = []
    with open(os.path.join(golden_dir, "philox4x32_10_kat.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                v = [int(t, 16) for t in line.split()]
                rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


def test_known_answers(golden_dir):
    rows = _kat(golden_dir)
    assert len(rows) == 3
    for ctr, key, want in rows:
        assert oracle.philox4x32_10(ctr, key).tolist() == want


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_matches_rocrand_block_function(tmp_path):
    exe = tmp_path / "rr_philox"
    subprocess.check_call(["hipcc", "-O1", "--offload-arch=gfx950", "-o", str(exe),
                           os.path.join(HERE, "rocrand_philox_ref.cpp")], cwd=str(tmp_path))
    rng = np.random.default_rng(123)
    cases = rng.integers(0, 2**32, size=(200, 6), dtype=np.uint64).astype(np.uint32)
    # counters shaped like the simulator's: (cell, period, rep, tag)
    cases[:50, 1] = rng.integers(0, 72, 50)
    cases[:50, 3] = rng.integers(0, 5, 50)
    text = "\n".join(" ".join(f"{int(v):08x}" for v in row) for row in cases) + "\n"
    out = subprocess.run([str(exe)], input=text, capture_output=True, text=True, check=True).stdout
    got = [[int(t, 16) for t in line.split()] for line in out.strip().splitlines()]
    assert len(got) == len(cases)
    for row, ref in zip(cases, got):
        assert oracle.philox4x32_10(row[:4], row[4:6]).tolist() == ref
