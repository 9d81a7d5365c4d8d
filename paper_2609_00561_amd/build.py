"""Build libiccg.so in-tree for gfx950.

Host-only C++ (ordering, schedules, host IC(0)) is compiled with g++ and
-ffp-contract=off so the ordering arithmetic is reproducible; the HIP sources
are compiled with hipcc for gfx950 with packed-FP32 instructions disabled and
kernel arguments preloaded into scalar registers (the leading 56 bytes of a
launch's arguments are in registers when a wavefront starts; the kernels put
the arguments they read first at the front).

Run as ``python -m paper_2609_00561_amd.build``.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libiccg.so")

HOST_SOURCES = ["order.cpp", "setup.cpp"]
HIP_SOURCES = ["iccg.hip", "mpnn.hip"]
ARCH = os.environ.get("ICCG_OFFLOAD_ARCH", "gfx950")


def _run(cmd):
    print("+", " ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    for src in HOST_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        _run(["g++", "-O2", "-std=c++17", "-fPIC", "-ffp-contract=off", "-Wall", "-Wextra",
              "-I", INCLUDE, "-I", CSRC, "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    for src in HIP_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        _run(["hipcc", "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-mllvm", "-amdgpu-kernarg-preload-count=16",
              "-Wno-unused-command-line-argument",
              "-I", INCLUDE, "-I", CSRC, "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    tmp = LIB + ".tmp"
    _run(["hipcc", "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
