"""Build the FP64 CPU oracle (test infrastructure) into oracle/liboracle.so.

Plain gcc, double precision, no contraction of a*b+c into fused multiply-adds,
OpenMP over lattice rows.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    # A temporary name per process: parallel test workers build at once, and
    # each swaps its own complete library into place.
    tmp = f"{LIB}.{os.getpid()}.tmp"
    cmd = ["gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-fopenmp",
           "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra",
           "-o", tmp, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
