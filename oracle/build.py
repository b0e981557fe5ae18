"""Builds oracle/liboigks.so from igks_oracle.c with gcc (plain C99, -O2,
no fast-math, OpenMP for the optional threads of its per-cell and per-face
loops).  Test infrastructure: the GPU library does not link it."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "igks_oracle.c")
LIB = os.path.join(HERE, "liboigks.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c99", "-D_DEFAULT_SOURCE", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
           "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
