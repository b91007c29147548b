"""Compile the C oracles (D2Q9 and D3Q19) into ``oracle/liblbm_oracle.so`` (test infrastructure).

Plain ``gcc -O2`` with OpenMP, no fast-math and no floating-point contraction,
so the oracle evaluates its formulas in the order it writes them.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRCS = [os.path.join(HERE, "lbm_oracle.c"), os.path.join(HERE, "lbm3d_oracle.c")]
LIB = os.path.join(HERE, "liblbm_oracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
           "-ffp-contract=off", "-fno-fast-math", "-D_DEFAULT_SOURCE",
           "-Wall", "-Wextra", "-Wno-unused-parameter",
           *SRCS, "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
