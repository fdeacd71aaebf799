"""Compile the HIP libraries for gfx950, in-tree next to this file: liblbmib.so
(the lattice Boltzmann / immersed boundary path) and libhbmceiling.so (the
reference streaming kernels the path's bandwidth is compared with)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc", "lbm_ib.hip")
LIB = os.path.join(HERE, "liblbmib.so")
CEIL_SRC = os.path.join(HERE, "csrc", "hbm_ceiling.hip")
CEIL_LIB = os.path.join(HERE, "libhbmceiling.so")
HEADERS = [os.path.join(HERE, "csrc", h) for h in ("lattice.hpp", "env.hpp", "fluid.hpp", "ib.hpp", "batch.hpp", "step.hpp",
                                                   "adjoint.hpp", "swimmer.hpp")] + [
    os.path.join(ROOT, "include", "lbm_ib.h")]

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def _compile(src: str, lib: str, verbose: bool) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = lib + ".tmp"
    cmd = [hipcc] + HIPCC_FLAGS + [src, "-o", tmp]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    return lib


def build(verbose: bool = False) -> str:
    _compile(CEIL_SRC, CEIL_LIB, verbose)
    return _compile(SRC, LIB, verbose)


if __name__ == "__main__":
    build(verbose=True)
