"""Compile the oracle's C++ into oracle/_build/liboracle.so (g++, FP64 plus exact FP32 emulation).

Contraction of multiply-add pairs and fast-math are disabled so every FP32 step of the projection
rounds on its own, as the binning contract requires.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(OUT_DIR, "liboracle.so")


def build(verbose=False) -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    src = os.path.join(HERE, "oracle.cpp")
    tmp = LIB + ".tmp"
    cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-msse2", "-mfpmath=sse", "-fPIC", "-shared", "-Wall", "-o", tmp, src]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
