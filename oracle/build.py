"""Compile the CPU oracle (test infrastructure) into oracle/libfsgo.so.

Plain gcc, OpenMP, no floating-point contraction so that every operation
is the rounded FP64 operation written in the source.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libfsgo.so")


def build(verbose: bool = False) -> str:
    cmd = [
        "gcc", "-std=gnu99", "-O3", "-march=x86-64-v2", "-ffp-contract=off",
        "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
        os.path.join(HERE, "fsgo.c"), "-o", LIB + ".tmp", "-lm",
    ]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
