"""Build the CPU oracle shared library (test infrastructure only).

Compiled with plain gcc, -O2 -ffp-contract=off and no fast-math, so each
floating-point operation of the oracle is one IEEE binary64 operation in
source order.  -fopenmp enables the oracle's two thread-parallel loops
(bitwise the single-thread results; one thread unless asked).
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csk_oracle.c")
LIB = os.path.join(HERE, "libcsk_oracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
