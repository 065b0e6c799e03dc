"""Builds libslosh.so (the HIP kernels and the C ABI of include/slosh.h) for gfx950."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libslosh.so")
SOURCES = [os.path.join(PKG, "csrc", f) for f in ("sph.hip", "mlp.hip", "lpv.hip")]

FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         # packed FP32 instructions are kept out of every kernel
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         # MFMA accumulators in ordinary vector registers: the network
         # kernels' epilogues then read them without a copy out of the
         # accumulation registers (the SPH kernels have no MFMA)
         "-mllvm", "-amdgpu-mfma-vgpr-form",
         "-I", os.path.join(ROOT, "include")]


def build(verbose: bool = False) -> str:
    srcs = [s for s in SOURCES if os.path.exists(s)]
    tmp = LIB + ".tmp"
    cmd = ["/opt/rocm/bin/hipcc", *FLAGS, "-o", tmp, *srcs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed")
    if verbose:
        sys.stderr.write(r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
