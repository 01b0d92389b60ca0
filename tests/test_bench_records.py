"""The measured HBM traffic that bench.py reports belongs to the kernel
sources in the tree: every propagation profile under profiles/ and every
TRAFFIC entry name the current digest of the kernel sources, and the
traffic figures in the profiles equal bench.py's."""
import glob
import os
import re

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_traffic_entries_and_profiles_name_the_current_sources():
    digest = bench.kernel_digest()
    assert {v[0] for v in bench.TRAFFIC.values()} == {digest}
    files = sorted(glob.glob(os.path.join(ROOT, "profiles", "propagate_*.md")))
    assert files
    for f in files:
        m = re.search(r"Kernel sources digest ([0-9a-f]{16})", open(f).read())
        assert m and m.group(1) == digest, os.path.basename(f)


def test_profile_traffic_equals_bench_traffic():
    names = {"large-8192x8192-64reps-72h": "propagate_large_8192x8192_64reps_72h.md",
             "batched-mc-1024x1024-2048reps": "propagate_batched_mc_1024x1024_2048reps.md",
             "single-fire-2048x2048-48h": "propagate_single_fire_2048x2048_48h.md"}
    for workload, fname in names.items():
        text = open(os.path.join(ROOT, "profiles", fname)).read()
        m = re.search(r"Measured HBM traffic ([0-9,]+) B per launch", text)
        assert m, fname
        assert int(m.group(1).replace(",", "")) == bench.TRAFFIC[workload][1], fname
