"""Builds libbfsmi.so (the HIP library behind include/bfs.h) for gfx950.

hipcc cross-compiles for the GPU without one being present.  The library is
built in-tree, next to this file.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libbfsmi.so")
ARCH = os.environ.get("BFSMI_ARCH", "gfx950")

SOURCES = ["frontier.hip", "relabel.hip", "rowskip.hip", "msbfs.hip", "smallloop.hip",
           "msloop.hip", "api.hip", "noalloc.hip", "grid2d.hip", "bottomup.hip", "batch_api.hip", "server.cpp"]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]


def build(verbose: bool = False) -> str:
    """Compile every HIP/C++ source into libbfsmi.so (always recompiles)."""
    objs = []
    os.makedirs(os.path.join(HERE, "_build"), exist_ok=True)
    common = ["-O3", "-std=c++17", "-fPIC", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
              "-Wall", "-Wno-unused-result"]
    # the kernels aggregate their counter atomics per wave themselves; the
    # compiler's atomic rewrite would read each result back at once and
    # stall the expansion pipeline
    gpu = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-munsafe-fp-atomics", "-mllvm", "-amdgpu-atomic-optimizer-strategy=None"]
    procs = []
    for src in sources():
        obj = os.path.join(HERE, "_build", os.path.basename(src) + ".o")
        if src.endswith(".hip"):
            cmd = [hipcc()] + common + gpu + ["-c", src, "-o", obj]
        else:
            cmd = [hipcc()] + common + ["-pthread", "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), file=sys.stderr)
        procs.append((subprocess.Popen(cmd), src))
        objs.append(obj)
    for p, src in procs:
        if p.wait() != 0:
            raise RuntimeError("compilation failed: " + src)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", "-pthread", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
