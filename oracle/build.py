"""Compile the FP64 CPU oracle (test infrastructure) into oracle/liblbm_oracle.so.

The oracle is plain C built with gcc; it shares no source with the HIP
library.  -ffp-contract=off keeps every product rounded on its own so the
particle-node predicate rounds the same way as any other implementation.
-fopenmp runs its per-node loops over z-planes in parallel; its sums are
taken per plane in a fixed order, so the thread count does not change a bit
of the result.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm_oracle.c")
LIB = os.path.join(HERE, "liblbm_oracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-fopenmp", "-Wall", "-Wextra", "-Wno-unused-parameter",
           "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
