"""Build step for the HIP library (gfx950) and, for the test suite, the CPU oracle.

``python -m paper_1606_00545_amd.build`` compiles every ``csrc/*.hip`` file into
``libhec.so`` next to this file with hipcc for gfx950, and the host-only build
of the triangular-solve planner (``csrc/plan_cpu.cpp``) into ``libhecplan.so``,
which lets the test suite check solve plans without a GPU.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libhec.so")
PLAN_LIB = os.path.join(HERE, "libhecplan.so")
ARCH = "gfx950"


def hip_sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


HIPCC_FLAGS = [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
               # no packed-FP32 instructions anywhere in device code
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
OBJ_DIR = os.path.join(os.path.dirname(HERE), "_build")


def hipcc_command(out: str = LIB):
    """The whole library in one hipcc call (the same flags as the per-file build)."""
    return ["hipcc"] + HIPCC_FLAGS + ["-shared", "-o", out] + hip_sources()


def _obj(src):
    return os.path.join(OBJ_DIR, os.path.basename(src) + ".o")


def plan_command(out: str = PLAN_LIB):
    return ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-Wall", "-o", out,
            os.path.join(CSRC, "plan_cpu.cpp")]


def _run(cmd, out, verbose):
    tmp = out + ".tmp"
    cmd = [tmp if c == out else c for c in cmd]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)


def build_plan(verbose: bool = False) -> str:
    _run(plan_command(), PLAN_LIB, verbose)
    return PLAN_LIB


def build(verbose: bool = False) -> str:
    """Compiles every source file for gfx950 (in parallel, one hipcc per file) and links
    libhec.so; then the host build of the planner."""
    from concurrent.futures import ThreadPoolExecutor
    os.makedirs(OBJ_DIR, exist_ok=True)
    srcs = hip_sources()

    def compile_one(src):
        cmd = ["hipcc"] + HIPCC_FLAGS + ["-c", "-o", _obj(src), src]
        if verbose:
            print(" ".join(cmd), flush=True)
        return subprocess.run(cmd, capture_output=True, text=True)

    with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        results = list(ex.map(compile_one, srcs))
    for src, r in zip(srcs, results):
        out = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l)
        if out.strip():
            print(out, flush=True)
        if r.returncode != 0:
            raise subprocess.CalledProcessError(r.returncode, f"hipcc -c {src}")
    _run(["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", LIB] + [_obj(s) for s in srcs], LIB, verbose)
    build_plan(verbose)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
