"""Build step for the HIP library: compiles ``csrc/*.hip`` for gfx950 into
``paper_1705_01022_amd/lib/libokpz.so`` with hipcc (cross-compiles without a GPU).

Usage: ``python -m paper_1705_01022_amd.build`` (or ``__graft_entry__.build()``).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC_DIR = os.path.join(HERE, "csrc")
LIB_DIR = os.path.join(HERE, "lib")
LIB = os.path.join(LIB_DIR, "libokpz.so")
ARCH = "gfx950"
SOURCES = ["okpz.hip", "batch.hip", "server.hip", "noalloc.hip"]

COMPILE_FLAGS = [
    "-O3",
    "-std=c++17",
    "--offload-arch=" + ARCH,
    "-fPIC",
    # no packed-FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # let the rounds of one Philox block unroll fully in the DB step kernel
    "-mllvm", "-pragma-unroll-threshold=200000",
    "-Wall",
    "-Wno-unused-function",
]


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP library cannot be built")


def build(verbose: bool = False) -> str:
    """Compile every source to an object in parallel, then link the library."""
    os.makedirs(LIB_DIR, exist_ok=True)
    tag = "%d" % os.getpid()
    objs, procs = [], []
    for f in SOURCES:
        obj = os.path.join(LIB_DIR, "%s.%s.o" % (os.path.splitext(f)[0], tag))
        cmd = [hipcc()] + COMPILE_FLAGS + ["-c", "-o", obj, os.path.join(SRC_DIR, f)]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True), f))
        objs.append(obj)
    failed = []
    for proc, f in procs:
        out, _ = proc.communicate()
        if proc.returncode != 0:
            sys.stderr.write(out)
            failed.append(f)
    try:
        if failed:
            raise RuntimeError("hipcc failed compiling %s" % ", ".join(failed))
        tmp = LIB + ".tmp" + tag
        cmd = [hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
        if verbose:
            print(" ".join(cmd), flush=True)
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError("hipcc failed linking %s" % LIB)
        os.replace(tmp, LIB)
    finally:
        for obj in objs:
            if os.path.exists(obj):
                os.remove(obj)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
