"""Build the HIP library libesi.so for gfx950 (MI355X) with hipcc."""
from __future__ import annotations

import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libesi.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # device code only: no value on the path can be NaN (integer times,
    # parameters checked finite on the host), so the clamps' min/max need no
    # canonicalised operands (one to two FP64 operations per event less)
    "-Xarch_device", "-fno-honor-nans",
    "-Wall", "-Wno-unused-result",
]
# named host ranges for profilers (roctx, ROCm's rocprofiler-sdk)
LINK_FLAGS = ["-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx"]


def sources():
    return sorted(glob.glob(os.path.join(PKG, "csrc", "*.hip")))


def build(out: str = LIB, verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    cmd = [hipcc, *HIPCC_FLAGS, "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(PKG, "csrc"), "-o", out + ".tmp", *sources(), *LINK_FLAGS]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
