"""Build libsor.so for gfx950 with hipcc (in place, next to this file).

Every HIP source is compiled with
  -ffp-contract=off      no multiply-add is fused unless the source asks for it,
                         so every rounding of the sweep is the one written (the
                         update's two fused steps are explicit fma calls);
  -Xclang -target-feature -Xclang -packed-fp32-ops
                         no packed FP32 instructions are generated.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libsor.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
    "-I" + os.path.join(ROOT, "include"),
]


def sources():
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")) +
                  glob.glob(os.path.join(HERE, "csrc", "*.cpp")))


def build(verbose: bool = False) -> str:
    objs = []
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    live = {os.path.basename(s) + ".o" for s in sources()}
    for f in os.listdir(objdir):
        if f not in live:
            os.remove(os.path.join(objdir, f))
    procs = []
    jobs = max(1, min(16, os.cpu_count() or 1))
    for src in sources():
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        lang = ["-x", "hip"]
        cmd = [HIPCC] + lang + [f for f in FLAGS if f not in ("-shared",)] + ["-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        while sum(p.poll() is None for p, _ in procs) >= jobs:
            time.sleep(0.05)
        procs.append((subprocess.Popen(cmd), src))
        objs.append(obj)
    bad = [src for p, src in procs if p.wait() != 0]
    if bad:
        raise RuntimeError(f"hipcc failed on {bad}")
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
