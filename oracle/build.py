"""Builds the oracle's shared library (liboracle.so) with the host C compiler.

The oracle is test infrastructure: plain C99, compiled without floating-point
contraction so that every product and sum is rounded on its own.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")


# -ffp-contract=off and -fno-fast-math: every product and sum rounded on its own
FLAGS = ["-std=c99", "-O3", "-ffp-contract=off", "-fno-fast-math"]


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "oracle.c")
    cmd = (["gcc"] + FLAGS + ["-fPIC", "-shared", "-Wall", "-Wextra", "-Wno-unused-parameter", "-o", LIB + ".tmp",
                              src, "-lm"])
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True, cwd=HERE)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
