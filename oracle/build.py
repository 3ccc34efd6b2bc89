"""Build the CPU oracle shared library (test infrastructure only).

The oracle is plain FP64 C++ compiled with no fast-math and no FMA contraction,
so its arithmetic is ordinary IEEE double in source order.  OpenMP only spreads
independent lines and cells over threads; it never changes the order of any sum.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm_oracle.cpp")
LIB = os.path.join(HERE, "liblbm_oracle.so")


def build(force: bool = True) -> str:
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared",
           "-ffp-contract=off", "-fno-fast-math", "-Wall", "-o", LIB + ".tmp", SRC]
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build())
