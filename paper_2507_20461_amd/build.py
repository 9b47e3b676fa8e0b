"""Build step of the HIP library (hipcc for gfx950, in-tree shared object)."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
SRC = os.path.join(PKG, "csrc", "geno_gks.hip")
SRCS = [SRC, os.path.join(PKG, "csrc", "opcount.hip"), os.path.join(PKG, "csrc", "mlp.hip"),
        os.path.join(PKG, "csrc", "geno6.hip"), os.path.join(PKG, "csrc", "geno_tri.hip")]
HEADERS = [os.path.join(PKG, "csrc", h) for h in ("geno_device.hpp", "gks_device.hpp", "mlp_device.hpp",
                                                  "geno6_device.hpp")] + [
    os.path.join(ROOT, "include", h) for h in ("geno_gks.h", "geno6.h", "geno_tri.h")]
LIB = os.path.join(PKG, "libgeno_gks.so")
ARCH = "gfx950"

FLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-shared",
    # contract a*b+c into FMA only within one expression, so that the x and y
    # instantiations of a kernel round identically (bitwise transpose symmetry)
    "-ffp-contract=on",
    "-I" + os.path.join(ROOT, "include"),
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def build(extra=(), verbose=False) -> str:
    """Compile the library (always recompiles)."""
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["/opt/rocm/bin/hipcc", *FLAGS, *extra, "-o", tmp, *SRCS]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(p) > t for p in [*SRCS, *HEADERS])


if __name__ == "__main__":
    build(extra=sys.argv[1:], verbose=True)
    print(LIB)
