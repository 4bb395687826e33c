"""Builds the CPU oracle library (test infrastructure only).

The oracle is plain C compiled by gcc with OpenMP.  IEEE semantics are kept
(-ffp-contract=off, no fast-math) so that its arithmetic is exactly what the
source says.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "hpgmx_oracle.c")
LIB = os.path.join(HERE, "libhpgmx_oracle.so")


def build_oracle(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
           "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wno-unused-function",
           "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build_oracle(verbose=True))
    sys.exit(0)
