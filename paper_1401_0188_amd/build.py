"""Build liblbm13.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_1401_0188_amd.build   (or __graft_entry__.build()).
Extra preprocessor definitions can be passed as arguments (-DNAME=VALUE).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbm13.so")
SOURCES = [os.path.join(CSRC, "lbm13_kernels.hip"), os.path.join(CSRC, "lbm13_capi.cpp"),
           os.path.join(CSRC, "lbm13_tune_cache.cpp")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# -packed-fp32-ops: no packed FP32 VALU instructions are generated.
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(ROOT, "include")]


def build(extra=(), out: str = LIB, verbose: bool = False) -> str:
    objs = []
    build_dir = os.path.join(HERE, "_build")
    os.makedirs(build_dir, exist_ok=True)
    for src in SOURCES:
        obj = os.path.join(build_dir, os.path.basename(src) + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmd = [HIPCC] + FLAGS + list(extra) + lang + ["-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


EXAMPLE_SRC = os.path.join(HERE, "examples", "c_api_example.cpp")
EXAMPLE = os.path.join(HERE, "examples", "c_api_example")


def build_example(out: str = EXAMPLE, verbose: bool = False) -> str:
    """Compile the standalone C-ABI example against the built library (no
    PyTorch): hipMalloc'd workspace, the library's calls, a decay check."""
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-O2", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", "-I" + os.path.join(ROOT, "include"), EXAMPLE_SRC,
           "-L" + HERE, "-llbm13", "-Wl,-rpath," + HERE, "-Wl,-rpath,$ORIGIN/..", "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(extra=sys.argv[1:], verbose=True))
    print(build_example(verbose=True))
