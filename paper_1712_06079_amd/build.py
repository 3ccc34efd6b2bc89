"""Build the HIP library for gfx950 in-tree: paper_1712_06079_amd/liblbm_hip.so.

Every HIP translation unit is compiled with packed FP32 instructions disabled
(-Xclang -target-feature -Xclang -packed-fp32-ops).  clang forwards that cc1
option to the host pass of a .hip file too (a driver option with arguments
cannot be restricted to the device pass), where the host backend reports the
feature as unknown and ignores it: those notes are dropped from the output.
The pure host sources (.cpp) are compiled by the host compiler without it.
Objects are built in parallel under _build/ and linked by hipcc.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "liblbm_hip.so")
HIP_SOURCES = ["lbm_api.hip", "lbm_batch.hip", "lbm_probe.hip"]
HOST_SOURCES = ["eos_host.cpp", "hdm_coeffs.cpp", "interface_host.cpp"]
SOURCES = HIP_SOURCES + HOST_SOURCES
HEADERS = ["lbm_device.hpp", "lbm_kernels.hpp", "lbm_fused.hpp", "lbm_march.hpp", "lbm_adjoint.hpp", "lbm_internal.hpp", "eos_host.hpp", "hdm_coeffs.hpp", "interface_host.hpp"]
ARCH = os.environ.get("LBM_OFFLOAD_ARCH", "gfx950")
NO_PACKED_FP32 = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
HOST_NOTE = "'-packed-fp32-ops' is not a recognized feature for this target"


def hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.isabs(c) and os.path.exists(c) or not os.path.isabs(c)):
            return c
    return "hipcc"


def _obj(src):
    return os.path.join(OBJ, os.path.splitext(src)[0] + ".o")


def compile_commands():
    inc = ["-I", os.path.join(ROOT, "include")]
    cmds = []
    for s in HIP_SOURCES:
        cmds.append([hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-c"] + NO_PACKED_FP32 + inc +
                    ["-o", _obj(s), os.path.join(CSRC, s)])
    for s in HOST_SOURCES:
        cmds.append(["g++", "-O3", "-std=c++17", "-fPIC", "-c"] + inc + ["-o", _obj(s), os.path.join(CSRC, s)])
    return cmds


def link_command(out=LIB):
    return [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", out] + [_obj(s) for s in SOURCES]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    lines = [ln for ln in (r.stdout + r.stderr).splitlines() if HOST_NOTE not in ln and "--hip-link" not in ln]
    if lines:
        print("\n".join(lines), file=sys.stderr, flush=True)
    if r.returncode != 0:
        raise subprocess.CalledProcessError(r.returncode, cmd)


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        for f in [ex.submit(_run, c, verbose) for c in compile_commands()]:
            f.result()
    tmp = LIB + ".tmp"
    _run(link_command(tmp), verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
