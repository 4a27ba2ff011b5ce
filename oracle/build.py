"""Build the FP64 CPU oracle library (test infrastructure only).

``python -m oracle.build`` compiles ``btdf_oracle.c`` into
``liboracle_btdf.so`` beside it with gcc. FMA contraction is off so the
oracle rounds every product and sum as the plain C expression reads; the
target stays generic x86-64 so the library runs on any host it is copied to.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "btdf_oracle.c")
LIB = os.path.join(HERE, "liboracle_btdf.so")


def build(verbose: bool = False) -> str:
    cmd = [
        "gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-fopenmp",
        "-ffp-contract=off", "-fno-fast-math", "-D_GNU_SOURCE",
        "-Wall", "-Wextra", "-Wno-unused-parameter",
        SRC, "-o", LIB + ".tmp", "-lm",
    ]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
