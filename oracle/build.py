"""Compile the CPU oracle (plain C, FP64) into oracle/liboracle.so.

Test infrastructure only.  gcc, no fast-math and no FMA contraction, so each
floating-point operation in the source is one IEEE operation.  OpenMP is linked
for the threaded timing mode (orc_set_threads); the default is one thread.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "rapdhg_oracle.c")
OUT = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c99", "-D_POSIX_C_SOURCE=199309L", "-ffp-contract=off",
           "-fno-fast-math", "-fopenmp", "-Wall", "-Wextra", "-fPIC", "-shared", "-o", OUT + ".tmp", SRC,
           "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(OUT)
