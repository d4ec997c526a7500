"""Build step for the CPU oracle (test infrastructure): compiles ugks_oracle.c with gcc.

Plain FP64: -O2 -ffp-contract=off, no fast math; OpenMP over rows (each cell's arithmetic
is the same at any thread count).
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ugks_oracle.c")
LIB = os.path.join(HERE, "libugks_oracle.so")


def build_oracle(verbose=False):
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
           "-shared", "-std=c11", "-D_DEFAULT_SOURCE", "-Wall", "-Wextra", SRC, "-o", tmp,
           "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build_oracle(verbose=True))
