"""Build the gfx950 HIP library libclb.so in-tree with hipcc."""
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libclb.so")
SOURCES = [os.path.join(CSRC, f) for f in
           ("clb_kernels.hip", "clb_state.hip", "nn_kernels.hip", "clb_api.cpp")]
ARCH = os.environ.get("CLB_OFFLOAD_ARCH", "gfx950")

# Packed FP32 instructions are disabled for all device code.
HIPFLAGS = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(verbose: bool = False, extra=()) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    cmd = [hipcc, "--offload-arch=" + ARCH, *HIPFLAGS, *extra, "-shared",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-o", LIB + ".tmp", *SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
