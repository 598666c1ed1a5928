"""Compile the HIP library (libwtree.so) in-tree for gfx950 with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libwtree.so")
CHECK_LIB = os.path.join(PKG, "libwtree_check.so")  # the write-counting build (WT_WRITE_CHECK)
SOURCES = ["wt_build.hip", "wt_small.hip", "wt_query.hip", "wt_buffered.hip", "wt_multiary.hip", "wt_huffman.hip", "wt_quad.hip",
           "wt_api.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-function",
]


CPU_SRC = os.path.join(PKG, "cpu", "wt_cpu.c")
CPU_LIB = os.path.join(PKG, "libwtcpu.so")


def build_cpu(verbose: bool = False) -> str:
    """The multicore CPU comparator (OpenMP), a separate host library."""
    tmp = CPU_LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", tmp, CPU_SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, CPU_LIB)
    return CPU_LIB


def build(verbose: bool = False, check: bool = False) -> str:
    """Compile every source to an object in parallel (one hipcc per file; each
    file launches only its own kernels, so no relocatable device code is
    needed), then link the shared library.  check: the write-counting build
    (WT_WRITE_CHECK, libwtree_check.so) instead of the product one."""
    import tempfile
    from concurrent.futures import ThreadPoolExecutor

    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    cflags = [f for f in FLAGS if f != "-shared"] + (["-DWT_WRITE_CHECK"] if check else [])
    out = CHECK_LIB if check else LIB
    with tempfile.TemporaryDirectory(prefix="wtree_build_") as tmpdir:
        objs, cmds = [], []
        for s in SOURCES:
            obj = os.path.join(tmpdir, s.replace(".hip", ".o"))
            objs.append(obj)
            cmds.append([HIPCC, *cflags, *inc, "-c", "-o", obj, os.path.join(CSRC, s)])

        def run(cmd):
            if verbose:
                print(" ".join(cmd), flush=True)
            subprocess.check_call(cmd)

        workers = max(1, min(len(cmds), os.cpu_count() or 1, 16))
        with ThreadPoolExecutor(max_workers=workers) as ex:
            for f in [ex.submit(run, c) for c in cmds]:
                f.result()
        tmp = out + ".tmp%d" % os.getpid()
        link = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
        run(link)
        os.replace(tmp, out)
    return out


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    build(verbose="-v" in sys.argv, check=True)
    build_cpu(verbose="-v" in sys.argv)
    print(LIB)
    print(CPU_LIB)
