"""Build the library's shared object in-tree (gfx950 device code, host C++).

Host sources (exact mesh/RNG arithmetic) are compiled by g++ with
-ffp-contract=off; device sources by hipcc for gfx950 with packed FP32
instructions disabled.  The result is ``liblfltsmc.so`` next to this file.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INC = os.path.join(ROOT, "include")
OUT = os.path.join(PKG, "liblfltsmc.so")
BUILD = os.path.join(PKG, "_build")

HOST_SRC = ["host_mesh.cpp", "host_rng.cpp", "host_line.cpp", "host_tri.cpp"]
DEV_SRC = ["lts_api.hip", "lts_step.hip", "lts_fused.hip", "lts_adjoint.hip", "lts_mlmc.hip", "lts_batch.hip", "lts_noalloc.hip", "lts_line.hip", "lts_tri.hip", "lts_mlts.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"


def _run(cmd):
    print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    for src in HOST_SRC:
        obj = os.path.join(BUILD, src + ".o")
        _run(["g++", "-O2", "-fPIC", "-std=c++17", "-ffp-contract=off", "-fno-builtin", "-Wall", "-I", INC, "-I", CSRC,
              "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    for src in DEV_SRC:
        obj = os.path.join(BUILD, src + ".o")
        _run([HIPCC, f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-I", INC, "-I", CSRC, "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    tmp = OUT + ".tmp"
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs)
    shutil.move(tmp, OUT)
    return OUT


if __name__ == "__main__":
    build()
    sys.exit(0)
