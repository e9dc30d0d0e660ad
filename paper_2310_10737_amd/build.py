"""Builds libsogrand.so (HIP, gfx950) in-tree with hipcc.

Each source compiles to its own object (in parallel), and the objects link into
one shared library.  The sources share no device symbols across files, so no
relocatable device code is needed.
"""
from __future__ import annotations

import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsogrand.so")
# the same library with per-phase wave clocks in the decode (SG_PHASE_CLOCKS), a measurement
# build that `bench.py --workload phases` loads instead of the product library
CLOCKED_LIB = os.path.join(HERE, "libsogrand_clocked.so")
OBJDIR = os.path.join(ROOT, "_build")

SOURCES = ["code.hip", "decode.hip", "batched.hip", "serve.hip", "profile.hip"]

HIPCC = "/opt/rocm/bin/hipcc"
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
    # packed FP32 VALU forms stay off: the compiler would otherwise emit them from
    # scalar float code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"),
]


# The persistent kernel loops over words: with machine-level loop-invariant code motion
# the compiler materialises the decode's constants once, before that loop, and keeps them
# in registers across every word, which costs resident waves.
SOURCE_FLAGS = {"batched.hip": ["-mllvm", "-disable-machine-licm"]}


def _compile(src: str, verbose: bool, clocked: bool = False) -> str:
    objdir = os.path.join(OBJDIR, "clocked") if clocked else OBJDIR
    obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
    extra = ["-DSG_PHASE_CLOCKS"] if clocked else []
    cmd = [HIPCC] + FLAGS + SOURCE_FLAGS.get(src, []) + extra + ["-c", "-o", obj, os.path.join(CSRC, src)]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    return obj


def build(verbose: bool = False, clocked: bool = False) -> str:
    """Compile every HIP source of the library and link them into one shared object (with
    clocked, the measurement build with per-phase wave clocks)."""
    os.makedirs(os.path.join(OBJDIR, "clocked") if clocked else OBJDIR, exist_ok=True)
    workers = max(1, min(len(SOURCES), len(os.sched_getaffinity(0))))
    with ThreadPoolExecutor(workers) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, clocked), SOURCES))
    lib = CLOCKED_LIB if clocked else LIB
    tmp = lib + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs + ["-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    import sys
    print(build(verbose=True, clocked="--phase-clocks" in sys.argv[1:]))
