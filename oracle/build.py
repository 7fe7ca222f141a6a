"""Compile the CPU oracle (test infrastructure) into oracle/libsphfilt_oracle.so.

Plain gcc, -O2, OpenMP over lines, FMA contraction off and no fast-math, so the
oracle's arithmetic is the textbook sum it is written as.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sphfilt_oracle.c")
LIB = os.path.join(HERE, "libsphfilt_oracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-Wextra", "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
