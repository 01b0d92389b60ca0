"""Build libc2f.so (gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libc2f.so")
SOURCES = ["prep.hip", "propagate.hip", "order.hip", "metrics.hip", "noalloc.hip", "account.hip", "capi.cpp"]
HEADERS = ["device.h", "fuel_table.h", "kernels.h", "ln64.h", "types.h"]

HIPCC_FLAGS = [
    "-std=c++17", "-O3", "-fPIC", "--offload-arch=gfx950",
    # keep packed-FP32 instructions out of all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # identical rounding of the rate arithmetic in every kernel that inlines it
    "-ffp-contract=off",
    "-Wall", "-Wno-unused-result", "-Wno-unused-command-line-argument",
]


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.isabs(cand) and os.path.exists(cand) or not os.path.isabs(cand)):
            return cand
    return "hipcc"


def build(verbose: bool = False) -> str:
    """Compile every source and link libc2f.so; always rebuilds."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    hipcc = _hipcc()
    objs = []
    env = dict(os.environ)
    env.setdefault("TMPDIR", "/tmp")
    procs = []
    for src in SOURCES:
        obj = os.path.join(objdir, src + ".o")
        cmd = [hipcc, *HIPCC_FLAGS, "-I", os.path.join(HERE, "..", "include"), "-c",
               os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), file=sys.stderr)
        # the sources compile independently: one compiler process each
        procs.append((src, subprocess.Popen(cmd, env=env, cwd=objdir)))
        objs.append(obj)
    failed = [src for src, p in procs if p.wait() != 0]
    if failed:
        raise subprocess.CalledProcessError(1, f"hipcc {' '.join(failed)}")
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs, "-lpthread"]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.run(cmd, check=True, env=env, cwd=objdir)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
