"""Builds librbsog.so in-tree: host C++ with g++ (-ffp-contract=off, the
sampling tables are fixed IEEE expression sequences), HIP sources with hipcc for
gfx950 only, linked into one shared library next to this file.  Also builds
libprice.so, the benchmark's measurement of FP64 elementary-function issue
costs (not part of the force path)."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
OUT = os.path.join(HERE, "librbsog.so")
PRICE_OUT = os.path.join(HERE, "libprice.so")
BUILD = os.path.join(HERE, "_build")

HOST_SRCS = ["host_sog.cpp", "host_tables.cpp", "host_near.cpp"]
HIP_SRCS = ["k_cells.hip", "k_sample.hip", "k_rho.hip", "k_near.hip", "k_far.hip", "api.hip", "ensemble.hip",
            "noalloc.hip", "observe.hip", "k_bath.hip"]

HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-ffp-contract=off", "-fno-fast-math", "-Wall", f"-I{INCLUDE}"]
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
             "-packed-fp32-ops", f"-I{INCLUDE}", "-Wall", "-Wno-unused-function"]


def _hipcc() -> str:
    for c in ("/opt/rocm/bin/hipcc", shutil.which("hipcc") or ""):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    for src in HOST_SRCS:
        obj = os.path.join(BUILD, src + ".o")
        subprocess.run(["g++", *HOST_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj], check=True)
        objs.append(obj)
    hipcc = _hipcc()
    for src in HIP_SRCS:
        obj = os.path.join(BUILD, src + ".o")
        cmd = [hipcc, *HIP_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), file=sys.stderr)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = OUT + ".tmp"
    subprocess.run([hipcc, "-shared", "--offload-arch=gfx950", "-o", tmp, *objs], check=True)
    os.replace(tmp, OUT)
    tmp = PRICE_OUT + ".tmp"
    subprocess.run([hipcc, *HIP_FLAGS, "-shared", os.path.join(CSRC, "price.hip"), "-o", tmp], check=True)
    os.replace(tmp, PRICE_OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
