"""Build the FP64 CPU oracle (test infrastructure) into ``oracle/libmppi_oracle.so``.

IEEE double precision, no fast-math and no FMA contraction, so that the oracle is
reproducible; OpenMP only parallelises the independent per-sample loop.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mppi_oracle.c")
LIB = os.path.join(HERE, "libmppi_oracle.so")


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fno-fast-math",
           "-ffp-contract=off", "-fopenmp", "-Wall", "-Wextra", "-o", tmp, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
