"""Build the HIP library for gfx950 in-tree: paper_1712_06079_amd/liblbm_hip.so.

Packed FP32 instructions are disabled for the device code (-packed-fp32-ops);
nothing else departs from hipcc -O3 defaults.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbm_hip.so")
SOURCES = ["lbm_api.hip", "lbm_batch.hip", "eos_host.cpp", "hdm_coeffs.cpp"]
HEADERS = ["lbm_device.hpp", "lbm_kernels.hpp", "lbm_fused.hpp", "lbm_march.hpp", "lbm_adjoint.hpp", "lbm_internal.hpp", "eos_host.hpp", "hdm_coeffs.hpp"]
ARCH = os.environ.get("LBM_OFFLOAD_ARCH", "gfx950")


def hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.isabs(c) and os.path.exists(c) or not os.path.isabs(c)):
            return c
    return "hipcc"


def command(out=LIB):
    return [hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(ROOT, "include"), "-o", out] + [os.path.join(CSRC, s) for s in SOURCES]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = command(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
