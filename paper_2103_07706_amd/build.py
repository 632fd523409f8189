"""Build libpa.so (HIP, gfx950) in place.

Every HIP source is compiled for gfx950 with packed FP32 instructions turned
off (-packed-fp32-ops); the host sources go through hipcc as well so that a
single shared object carries both.
"""
from __future__ import annotations

import glob
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(HERE, "libpa.so")


def build(verbose: bool = False) -> str:
    srcs = sorted(glob.glob(os.path.join(HERE, "csrc", "*.cpp")) +
                  glob.glob(os.path.join(HERE, "csrc", "*.hip")))
    tmp = SO + ".tmp"
    cmd = ["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
           "-shared", "-Wall", "-Wno-unused-result",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-o", tmp] + srcs
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, SO)
    return SO


if __name__ == "__main__":
    print(build(verbose=True))
