"""Compile the HIP library libtdse.so in-tree for gfx950.

    python -m paper_2001_06113_amd.build        (or build() from Python)

hipcc cross-compiles without a GPU.  Every HIP translation unit is built with
packed FP32 instructions disabled.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libtdse.so")

HIP_SOURCES = ["periodic_kernels.hip", "freespace_kernels.hip", "batch_fp64.hip", "batch_split.hip",
               "adjoint_kernels.hip", "far_kernels.hip", "run1d_kernels.hip", "persist2d_kernels.hip",
               "diag_kernels.hip"]
HOST_SOURCES = ["tdse_api.cpp"]
ARCH = os.environ.get("TDSE_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False, jobs: int = 4) -> str:
    """Compile every source to an object, then link libtdse.so.  Always rebuilds."""
    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    cc = hipcc()
    common = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function", "-Wno-unused-lambda-capture",
              f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}"]
    dev = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-ffp-contract=fast", "-munsafe-fp-atomics"]
    cmds, objs = [], []
    for src in HIP_SOURCES:
        obj = os.path.join(objdir, src + ".o")
        cmds.append([cc, *common, *dev, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    for src in HOST_SOURCES:
        obj = os.path.join(objdir, src + ".o")
        cmds.append([cc, *common, *dev, "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    # each compiler writes to its own log file (a pipe could fill up and stall it)
    procs = []
    for cmd, obj in zip(cmds, objs):
        if verbose:
            print(" ".join(cmd), flush=True)
        while sum(p.poll() is None for _, p, _ in procs) >= jobs:
            next(p for _, p, _ in procs if p.poll() is None).wait()
        log = open(obj + ".log", "w")
        procs.append((cmd, subprocess.Popen(cmd, stdout=log, stderr=subprocess.STDOUT), log))
    for cmd, p, log in procs:
        p.wait()
        log.close()
        out = open(log.name).read()
        if p.returncode != 0:
            raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{out[-8000:]}")
        if verbose and out.strip():
            print(out)
    tmp = LIB + ".tmp"
    link = [cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(link, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(link)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
