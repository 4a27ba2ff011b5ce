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


# the oracle built with AddressSanitizer and UndefinedBehaviorSanitizer:
# tests load it with ORACLE_LIBRARY and gcc's runtime (san_runtime) preloaded
SAN_LIB = os.path.join(HERE, "liboracle_btdf_san.so")


def san_runtime() -> str:
    out = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(out) or not os.path.exists(out):
        raise RuntimeError("no AddressSanitizer runtime found for gcc")
    return out


def build(verbose: bool = False, sanitize: bool = False) -> str:
    out = SAN_LIB if sanitize else LIB
    san = ["-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-fno-omit-frame-pointer"] if sanitize else []
    cmd = [
        "gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-fopenmp",
        "-ffp-contract=off", "-fno-fast-math", "-D_GNU_SOURCE",
        "-Wall", "-Wextra", "-Wno-unused-parameter",
    ] + san + [SRC, "-o", out + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    build(verbose="-v" in sys.argv, sanitize="--sanitize" in sys.argv)
