"""Compile the FP64 CPU oracle (test infrastructure) into oracle/liboracle.so.

Plain gcc, no GPU toolchain. ``-ffp-contract=off`` keeps every product and sum
rounded exactly as written in the C source. No ``-march=native``: the library
built here also runs on the benchmark machine's host, whose CPU may differ.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm_oracle.c")
OUT = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False, src: str = SRC, out: str = OUT) -> str:
    cmd = [
        "gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
        "-ffp-contract=off", "-Wall", "-Wextra", "-Wno-unused-parameter",
        "-o", out + ".tmp", src, "-lm",
    ]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
