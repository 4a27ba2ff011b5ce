"""Build ``libbtdf.so`` (the gfx950 HIP library behind include/btdf.h) in-tree.

``python -m paper_1806_09403_amd.build`` compiles every ``csrc/*.hip`` with
hipcc for gfx950 into ``paper_1806_09403_amd/libbtdf.so``.
"""
import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libbtdf.so")
ARCH = "gfx950"


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return "hipcc"


def flags():
    return [
        "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
        # packed FP32 instructions stay off (compiler-generated ones included)
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wall", "-Wno-unused-function", "-Wno-unused-result",
        "-I" + INCLUDE, "-I" + CSRC,
    ]


# the host code built with AddressSanitizer and UndefinedBehaviorSanitizer
# (device code is built as usual): tests load it with BTDF_LIBRARY and the
# runtime of SAN_RUNTIME preloaded
SAN_LIB = os.path.join(PKG, "_build", "san", "libbtdf_san.so")
SAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]


def san_runtime() -> str:
    """The compiler's shared AddressSanitizer runtime (to preload)."""
    out = subprocess.run([hipcc(), "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True,
                         text=True).stdout.strip()
    if not os.path.isabs(out) or not os.path.exists(out):
        found = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
        out = found[-1] if found else ""
    if not out:
        raise RuntimeError("no AddressSanitizer runtime found for hipcc")
    return out


def build(verbose: bool = False, sanitize: bool = False) -> str:
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    objs = []
    build_dir = os.path.join(PKG, "_build", "san") if sanitize else os.path.join(PKG, "_build")
    out = SAN_LIB if sanitize else LIB
    extra = (["-O1", "-g"] + SAN_HOST) if sanitize else []
    os.makedirs(build_dir, exist_ok=True)
    procs = []
    for s in srcs:
        o = os.path.join(build_dir, os.path.basename(s) + ".o")
        cmd = [hipcc()] + flags() + extra + ["-c", s, "-o", o]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((cmd, subprocess.Popen(cmd)))
        objs.append(o)
    for cmd, p in procs:
        if p.wait() != 0:
            raise RuntimeError("compile failed: " + " ".join(cmd))
    link = [hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC"] + (
        SAN_HOST + ["-shared-libsan"] if sanitize else []) + objs + ["-o", out + ".tmp"]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    build(verbose="-v" in sys.argv, sanitize="--sanitize" in sys.argv)
