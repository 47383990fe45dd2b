"""Build step: compile the HIP library for gfx950 in-tree.

    python -m paper_2512_01283_amd.build

produces paper_2512_01283_amd/libpolrad.so from csrc/ with hipcc.  Packed
FP32 instructions are disabled for all device code, and FP64 atomics are
allowed to lower to the native global_atomic_add_f64.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpolrad.so")
ARCH = "gfx950"

SOURCES = ["kp_kernels.hip", "kp_api.cpp", "kp_denoiser.hip", "kp_dn_api.cpp"]

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-munsafe-fp-atomics",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
    "-I", os.path.join(ROOT, "include"),
]


CALIB_SOURCE = "kp_calib.hip"
CALIB_LIB = os.path.join(HERE, "libkpcalib.so")


def build_calib(verbose: bool = False) -> str:
    """The device-calibration library that bench.py loads (not the method)."""
    cmd = ["hipcc", *FLAGS, "-shared", "-x", "hip", os.path.join(CSRC, CALIB_SOURCE), "-o", CALIB_LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(CALIB_LIB + ".tmp", CALIB_LIB)
    return CALIB_LIB


def build(verbose: bool = False, extra=()) -> str:
    objs = []
    tmp = os.path.join(HERE, "_build")
    os.makedirs(tmp, exist_ok=True)
    for src in SOURCES:
        obj = os.path.join(tmp, src + ".o")
        cmd = ["hipcc", *FLAGS, *extra, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", LIB + ".tmp"]
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    build_calib(verbose="-v" in sys.argv)
    print(LIB)
    print(CALIB_LIB)
