"""Compile the HIP library for gfx950, in-tree (liblbmib.so next to this file)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc", "lbm_ib.hip")
LIB = os.path.join(HERE, "liblbmib.so")
HEADERS = [os.path.join(HERE, "csrc", h) for h in ("lattice.hpp", "env.hpp", "fluid.hpp", "ib.hpp", "batch.hpp",
                                                   "adjoint.hpp", "swimmer.hpp")] + [
    os.path.join(ROOT, "include", "lbm_ib.h")]

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp"
    cmd = [hipcc] + HIPCC_FLAGS + [SRC, "-o", tmp]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
