"""Build libcfh.so (the gfx950 HIP library) in-tree with hipcc."""
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "libcfh.so")
SOURCES = ["frame.cpp", "plan.cpp", "kernels.hip", "pass2_c128.hip", "pass2_c64.hip", "batch.hip", "batch2.hip",
           "calib.hip", "noalloc.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # uniform branch trees (the per-rotation body dispatch) stay unstructured:
    # structurizing them makes every body's outputs live through the whole
    # tree, which costs register copies and occupancy
    "-mllvm", "-structurizecfg-skip-uniform-regions=true",
    # keep sibling leaves of the body switches apart: sinking their common
    # instructions merges them into one leaf with selected operands
    "-mllvm", "-sink-common-insts=false",
    "-Wall", "-Wno-unused-function", "-Wno-unused-result",
    "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
]


def build(verbose: bool = False, extra=()) -> str:
    """Compile every source to an object in parallel, then link the library."""
    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    cmds = []
    for src in SOURCES:
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        cmds.append(([HIPCC, *FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj], obj))
    procs = []
    for cmd, _ in cmds:
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd))
    failed = [c for (c, _), p in zip(cmds, procs) if p.wait() != 0]
    if failed:
        raise subprocess.CalledProcessError(1, failed[0])
    tmp = OUT + ".tmp"
    link = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *[o for _, o in cmds], "-o", tmp]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
