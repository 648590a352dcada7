"""Build the gfx950 library libhrt.so in-tree with hipcc (and g++ for the
float64 host plan).  Usable as `python -m paper_1604_07651_amd.build`."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libhrt.so")
ARCH = "gfx950"

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
# Packed FP32 instructions are disabled for all device code.
DEVICE_FLAGS = ["-O3", f"--offload-arch={ARCH}", "-fPIC", "-std=c++17",
                "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                "-munsafe-fp-atomics", "-I", INCLUDE, "-I", CSRC]
# The host plan takes integer decisions from float64 comparisons: no FMA
# contraction there.
HOST_FLAGS = ["-O2", "-fPIC", "-std=c++17", "-ffp-contract=off", "-pthread",
              "-I", INCLUDE, "-I", CSRC]


def _run(cmd):
    print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    plan_o = os.path.join(BUILD, "plan.o")
    hrt_o = os.path.join(BUILD, "hrt.o")
    cxx = shutil.which("g++") or "g++"
    _run([cxx, *HOST_FLAGS, "-c", os.path.join(CSRC, "plan.cpp"), "-o", plan_o])
    _run([HIPCC, *DEVICE_FLAGS, "-c", os.path.join(CSRC, "hrt.hip"), "-o", hrt_o])
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", hrt_o, plan_o,
          "-pthread", "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
