"""Compile libdpsnn.so (HIP for gfx950) in-tree.

Flags that matter for the results:
  -ffp-contract=off                 no fused multiply-add contraction, so the
                                    binary32 neuron update is exactly the
                                    written sequence of roundings;
  -fno-gpu-flush-denormals-to-zero  binary32 subnormals are kept;
  -target-feature -packed-fp32-ops  no packed FP32 instructions.
"""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libdpsnn.so")
SOURCES = ["api.hip", "kernels.hip", "waves.hip", "tables.cpp"]
ARCH = os.environ.get("DPSNN_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def build(verbose: bool = False) -> str:
    cmd = [hipcc(), "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-shared",
           "-ffp-contract=off", "-fno-gpu-flush-denormals-to-zero",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Wall", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           "-o", LIB + ".tmp"] + [os.path.join(CSRC, s) for s in SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
