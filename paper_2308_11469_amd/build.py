"""Builds the HIP library ``libfk_helmholtz.so`` in-tree for gfx950.

Every source under ``csrc/`` is compiled by ``hipcc`` (HIP for the kernels,
HIP host API for the runtime) and linked into one shared library whose only
interface is the C ABI declared in ``include/fk_helmholtz.h``.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libfk_helmholtz.so")
SOURCES = ["fk_kernels.hip", "fk_problem.cpp", "fk_solver.cpp", "fk_engine.cpp", "fk_static.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("FK_OFFLOAD_ARCH", "gfx950")
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
         # packed FP32 instructions stay off: scalar FP32 code only
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         # multiply-adds are fused only within one expression, never across
         # statements: the path kernel is compiled per feature set, and every
         # variant must round an instance's arithmetic the same way
         "-ffp-contract=on",
         "-Wall", "-Wno-unused-function", "-I" + os.path.join(HERE, "..", "include")]
FLAGS += os.environ.get("FK_HIPCC_FLAGS", "").split()   # extra compiler options


def _compile(src):
    obj = os.path.join(BUILD, src + ".o")
    cmd = [HIPCC] + FLAGS + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(ln for ln in (r.stdout + r.stderr).splitlines()
                    if "packed-fp32-ops' is not a recognized feature" not in ln)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, out))
    return obj, out


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(4, os.cpu_count() or 1)) as ex:
        results = list(ex.map(_compile, SOURCES))
    for obj, out in results:
        if verbose and out.strip():
            print(out)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH] + [o for o, _ in results] + ["-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


def is_built():
    return os.path.exists(LIB)


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
