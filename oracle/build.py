"""Build the CPU oracle shared library (test infrastructure only).

gcc -O2 -ffp-contract=off: no fused multiply-add contraction and no fast-math, so
binary32/binary64 arithmetic follows IEEE round-to-nearest-even operation by
operation; the only fused operations are the explicit fma() calls of the logarithm.
-fopenmp only spreads the independent rows of network construction over host threads;
the simulation loop is single-threaded.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["rng.c", "network.c", "simulate.c"]
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-fopenmp", "-fPIC",
           "-shared", "-Wall", "-Wextra", "-Wno-unused-parameter", "-o", LIB + ".tmp"]
    cmd += [os.path.join(HERE, s) for s in SOURCES] + ["-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
