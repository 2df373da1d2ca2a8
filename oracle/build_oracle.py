"""Compile the plain FP64 CPU oracle (test infrastructure) into oracle/libpond_oracle.so.

g++ with -O2 and OpenMP; no -ffast-math, so every sum keeps the order written in
the source.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pond_oracle.cpp")
LIB = os.path.join(HERE, "libpond_oracle.so")


def build(verbose: bool = False, extra_flags=(), out: str = LIB) -> str:
    cmd = ["g++", "-std=c++17", "-O2", "-fopenmp", "-fPIC", "-shared", "-fno-fast-math",
           "-ffp-contract=off", *extra_flags, "-o", out + ".tmp", SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
