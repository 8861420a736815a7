"""Build the HSIM shared library (libhsim.so) for gfx950 with hipcc.

Every call compiles every source again (no caching), in parallel, and links
``libhsim.so`` next to this file.  Host C++ is compiled without floating
point contraction so that the hierarchy's distance arithmetic is plain IEEE
double; HIP device code disables packed FP32 instructions.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libhsim.so")
ARCH = os.environ.get("HSIM_OFFLOAD_ARCH", "gfx950")

HOST_SOURCES = ["mesh.cpp", "hierarchy.cpp", "order.cpp"]        # plain C++ (no HIP)
DEVICE_SOURCES = ["hsim.cpp", "kernels.hip", "build_dev.hip"]    # HIP runtime / kernels


def _hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _clangxx():
    for c in ("/opt/rocm/llvm/bin/clang++", shutil.which("clang++"), shutil.which("g++")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("no host C++ compiler found")


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("build step failed:\n" + " ".join(cmd) + "\n" + r.stdout)
    return r.stdout


def build(verbose=False, jobs=None):
    hipcc = _hipcc()
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    common = ["-O3", "-fPIC", "-std=c++17", "-I" + os.path.join(ROOT, "include"), "-Wall", "-Wno-unused-function"]
    cmds, objs = [], []
    for src in HOST_SOURCES:
        obj = os.path.join(objdir, src + ".o")
        cmds.append([_clangxx(), *common, "-fopenmp", "-ffp-contract=off", "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    for src in DEVICE_SOURCES:
        obj = os.path.join(objdir, src + ".o")
        omp = ["-fopenmp"] if src == "hsim.cpp" else []   # host loops of the level set-up
        cmds.append([hipcc, *common, *omp, "-x", "hip", f"--offload-arch={ARCH}", "-munsafe-fp-atomics",
                     "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                     "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    with cf.ThreadPoolExecutor(max_workers=jobs or min(8, len(cmds))) as ex:
        outs = list(ex.map(_run, cmds))
    if verbose:
        for o in outs:
            if o.strip():
                print(o)
    tmp = LIB + ".tmp"
    _run([hipcc, "-shared", "-fopenmp", f"--offload-arch={ARCH}", "-o", tmp, *objs,
          "-Wl,-rpath,/opt/rocm/lib/llvm/lib", "-Wl,-rpath,/opt/rocm/lib"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
