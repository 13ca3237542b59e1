"""Build the HIP library libgg.so for gfx950, in-tree.

Every source under csrc/ is compiled by hipcc into one shared object that
exports the C ABI declared in include/gg.h. Packed FP32 instructions are
disabled (-packed-fp32-ops): the kernels rely on scalar FP32 arithmetic.
"""
import os
import shutil
import subprocess
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OUT = os.path.join(PKG, "libgg.so")
ARCH = "gfx950"


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def command(out: str = OUT):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    return [hipcc, f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-function", "-Wno-unused-result",
            "-I", INCLUDE, "-I", CSRC, "-o", out] + sources()


def build(verbose: bool = False) -> str:
    cmd = command(OUT + ".tmp")
    t0 = time.time()
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(OUT + ".tmp", OUT)
    if verbose:
        print(f"built {OUT} in {time.time() - t0:.1f} s", flush=True)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
