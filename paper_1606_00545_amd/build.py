"""Build step for the HIP library (gfx950) and, for the test suite, the CPU oracle.

``python -m paper_1606_00545_amd.build`` compiles every ``csrc/*.hip`` file into
``libhec.so`` next to this file with hipcc for gfx950.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libhec.so")
ARCH = "gfx950"


def hip_sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def hipcc_command(out: str = LIB):
    return (["hipcc", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
             "-Wall", "-Wno-unused-function",
             # no packed-FP32 instructions anywhere in device code
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-o", out] + hip_sources())


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = hipcc_command(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
