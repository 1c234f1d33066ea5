"""Build the CPU oracle shared library (test infrastructure only).

    python oracle/build_oracle.py

compiles ``sem_oracle.c`` with plain gcc, FP64, no fused multiply-add and no
fast-math, OpenMP over elements, into ``oracle/libsemoracle.so``.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libsemoracle.so")


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "sem_oracle.c")
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp",
           "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra",
           "-o", LIB + ".tmp", src, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
