"""Build the oracle's shared library with gcc (plain C, no FMA contraction, no fast-math; OpenMP
only for the row-parallel timing variant of the smoother)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    cmd = [
        "gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
        "-fopenmp", "-Wall", "-Wextra", "-Wno-unused-parameter",
        "-o", LIB, os.path.join(HERE, "oracle.c"), "-lm",
    ]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
