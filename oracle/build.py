"""Build the oracle shared library (plain C, FP64) with gcc.

Test infrastructure only: the product library never links it.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["philox.c", "linalg.c", "fd.c", "window.c", "attp.c", "p5.c", "cod.c"]
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False, src_dir: str = HERE, out: str = LIB) -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fno-fast-math",
           "-ffp-contract=off", "-I", HERE, "-o", out]
    cmd += [os.path.join(src_dir, s) for s in SOURCES]
    cmd += ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
