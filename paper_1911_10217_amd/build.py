"""Build librlc.so (HIP, gfx950) in-tree with hipcc.

Flags that the parity contract depends on:
  -ffp-contract=off                        no fused multiply-add contraction
  -fhip-fp32-correctly-rounded-divide-sqrt IEEE division and square root
  -fno-gpu-flush-denormals-to-zero         IEEE subnormals
  -Xclang -target-feature -Xclang -packed-fp32-ops   no packed FP32 ops
"""
from __future__ import annotations

import glob
import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "librlc.so")

ARCH = os.environ.get("RLC_OFFLOAD_ARCH", "gfx950")

DEVICE_FLAGS = [
    "-O3",
    "-std=c++17",
    "-ffp-contract=off",
    "-fhip-fp32-correctly-rounded-divide-sqrt",
    "-fno-gpu-flush-denormals-to-zero",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    for c in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def build(verbose: bool = False) -> str:
    """Compile every HIP source into librlc.so (always recompiles)."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = []
    cc = hipcc()
    for src in sources():
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        cmd = [cc, "--offload-arch=" + ARCH, "-fPIC", "-c", src, "-o", obj, "-I", INCLUDE, "-I", CSRC] + DEVICE_FLAGS
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [cc, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
