"""Build of the gfx950 HIP library (libporta.so) with hipcc, in-tree."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libporta.so")
HOSTTEST_LIB = os.path.join(PKG, "libporta_hostmath.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

# Packed FP32 instructions are disabled for all device code.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"build failed: {' '.join(cmd[:3])} ...")
    return r


def build_library(verbose: bool = False) -> str:
    srcs = [os.path.join(CSRC, "porta_abi.hip"), os.path.join(CSRC, "porta_see_mg.hip")]
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
           "-Wall", "-Wno-unused-result", "-I", os.path.join(ROOT, "include"), *DEVICE_FLAGS,
           *srcs, "-o", tmp]
    _run(cmd, verbose)
    os.replace(tmp, LIB)
    return LIB


def build_hostmath(verbose: bool = False) -> str:
    """Host build of the per-update arithmetic (porta_math.hpp) for CPU unit tests."""
    src = os.path.join(CSRC, "hostmath.cpp")
    tmp = HOSTTEST_LIB + ".tmp"
    cmd = [HIPCC, "-O2", "-std=c++17", "-fPIC", "-shared", "-x", "hip", "--offload-host-only",
           src, "-o", tmp]
    _run(cmd, verbose)
    os.replace(tmp, HOSTTEST_LIB)
    return HOSTTEST_LIB


def build_all(verbose: bool = False):
    return build_library(verbose), build_hostmath(verbose)


if __name__ == "__main__":
    print(build_all(verbose=True))
