"""Build the C-ABI shared library ``libfe_mi355x.so`` in-tree.

Host C++ (pattern, ordering, factorisation) is compiled with g++; HIP
sources with hipcc for gfx950; the library is linked with hipcc.  Objects go
to ``_build/`` next to this file.  ``python -m paper_2306_05893_amd.build``
builds from the command line.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libfe_mi355x.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")

HOST_SOURCES = ["host_pattern.cpp", "host_analyse.cpp", "host_factor.cpp", "host_gpuplan.cpp"]
HIP_SOURCES = ["kernels_element.hip", "kernels_solve.hip", "kernels_adjoint.hip",
               "kernels_factor.hip", "kernels_multi.hip", "kernels_guess.hip",
               "kernels_rotation.hip", "fe_api.hip"]

CXX = shutil.which("g++") or "g++"
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"

HOST_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-pthread", "-march=x86-64-v3", "-Wall",
              "-Wno-unused-function", f"-I{INCLUDE}"]
# packed FP32 instructions are disabled on purpose (see the design notes)
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-munsafe-fp-atomics",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             f"-I{INCLUDE}", "-Wno-unused-result"]


def _run(cmd):
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if p.returncode != 0:
        raise RuntimeError("build step failed:\n" + " ".join(cmd) + "\n" + p.stdout)
    return p.stdout


def build(verbose: bool = False, jobs: int = 8) -> str:
    os.makedirs(BUILD, exist_ok=True)
    cmds = []
    objs = []
    for src in HOST_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        cmds.append([CXX, *HOST_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    for src in HIP_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        cmds.append([HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        outs = list(ex.map(_run, cmds))
    if verbose:
        for c, o in zip(cmds, outs):
            print(" ".join(c))
            if o.strip():
                print(o)
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp, *objs, "-pthread"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
