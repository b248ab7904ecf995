"""Build the gfx950 shared library libec.so in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libec.so")
SOURCES = ["ec_stencil.hip", "ec_basis.hip", "ec_update.hip", "ec_adjoint.hip", "ec_static.hip",
           "ec_mass.hip", "ec_newton.hip", "ec_capi.cpp"]
ARCH = os.environ.get("EC_OFFLOAD_ARCH", "gfx950")


def hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.isabs(c) and os.path.exists(c) or not os.path.isabs(c)):
            return c
    return "hipcc"


def build(verbose=False):
    """Compile every HIP source into libec.so (always recompiles)."""
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
           # code object v5 loads under the HIP runtime that ships with torch
           "-mcode-object-version=5",
           # no packed FP32 (v_pk_*_f32) instructions
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           "-o", tmp] + [os.path.join(CSRC, s) for s in SOURCES] + [
           # roctx phase ranges (rocprofv3 --marker-trace)
           "-lrocprofiler-sdk-roctx"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
