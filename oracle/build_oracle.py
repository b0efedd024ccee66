"""Compile the plain C oracle into ``oracle/liboracle.so`` (test infrastructure).

The flags keep the arithmetic contract stated in ``oracle.c``: no fused
multiply-add contraction, no fast-math, IEEE division and square root.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

FLAGS = [
    "-O3", "-march=x86-64-v3", "-fPIC", "-shared", "-std=c11",
    "-ffp-contract=off", "-fno-fast-math", "-fno-unsafe-math-optimizations",
    "-fopenmp",
]


def build(verbose=False):
    cmd = ["gcc", *FLAGS, SRC, "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def ensure_built():
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        build()
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
