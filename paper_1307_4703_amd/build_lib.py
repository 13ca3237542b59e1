"""Build the HIP library libgg.so for gfx950, in-tree.

Every source under csrc/ is compiled by hipcc (in parallel, one object per
source under _build/) and linked into one shared object that exports the C
ABI declared in include/gg.h. Packed FP32 instructions are disabled
(-packed-fp32-ops): the kernels rely on scalar FP32 arithmetic.
"""
import os
import shutil
import subprocess
import sys
import time
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OUT = os.path.join(PKG, "libgg.so")
OBJ_DIR = os.path.join(ROOT, "_build")
ARCH = "gfx950"


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def hipcc():
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def flags():
    return [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-function", "-Wno-unused-result",
            "-I", INCLUDE, "-I", CSRC]


def command(out: str = OUT):
    """One hipcc command that compiles and links every source."""
    return [hipcc()] + flags() + ["-shared", "-o", out] + sources()


def build(verbose: bool = False, jobs: int = 0) -> str:
    t0 = time.time()
    os.makedirs(OBJ_DIR, exist_ok=True)
    srcs = sources()
    objs = [os.path.join(OBJ_DIR, os.path.basename(s) + ".o") for s in srcs]
    cmds = [[hipcc()] + flags() + ["-c", "-o", o, s] for s, o in zip(srcs, objs)]
    jobs = jobs or min(len(cmds), os.cpu_count() or 1, 8)

    def run(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)

    with ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(run, cmds))
    link = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", OUT + ".tmp"] + objs
    run(link)
    os.replace(OUT + ".tmp", OUT)
    if verbose:
        print(f"built {OUT} in {time.time() - t0:.1f} s", flush=True)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
