"""Build libgnorfdtd.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libgnorfdtd.so")
ARCH = os.environ.get("GNOR_OFFLOAD_ARCH", "gfx950")

COMMON = ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC",
          # packed-FP32 instructions stay off (plain scalar/vector float code only)
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I", os.path.join(os.path.dirname(HERE), "include")]

SOURCES = [
    ("gnor_sweeps.hip", []),
    ("gnor_fused.hip", []),
    ("gnor_fplain.hip", []),
    # matrix-core accumulators in ordinary VGPRs: with the accumulation
    # registers the loop-carried sums were copied out and back every step
    ("gnor_spectra.hip", ["-mllvm", "-amdgpu-mfma-vgpr-form=1"]),
    ("gnor_adjoint.hip", []),
    ("gnor_util.hip", []),
    # the voxelisers' floating-point tests must not be contracted into FMAs
    ("gnor_runtime.cpp", ["-ffp-contract=off"]),
]


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    for src, extra in SOURCES:
        obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
        cmd = ["hipcc", "-c", os.path.join(CSRC, src), "-o", obj] + COMMON + extra
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "-shared", "-o", tmp] + objs + [f"--offload-arch={ARCH}", "-fPIC"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
