"""Builds the C oracle (``liboracle_fkmc.so``) next to its source.

Test infrastructure only: see ``oracle/__init__.py``.  Plain ``gcc``, FP
contraction off, no fast-math, OpenMP over grid nodes.  ``-march=x86-64-v3``
keeps the library loadable on any AVX2 host, including hosts other than the
one that built it.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "fkmc.c")
LIB = os.path.join(HERE, "liboracle_fkmc.so")

CFLAGS = ["-O3", "-march=x86-64-v3", "-ffp-contract=off", "-fno-fast-math",
          "-fopenmp", "-Wall", "-Wextra", "-shared", "-fPIC"]


def build(verbose=False):
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc"] + CFLAGS + [SRC, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


def ensure_built():
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        build()
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
