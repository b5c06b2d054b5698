"""Build libkpm.so (all HIP sources under csrc/) for gfx950 with hipcc.

Usage: python -m paper_1910_05194_amd.build   (or build() from __graft_entry__)
Objects are compiled in parallel into csrc/_build/ and linked into
paper_1910_05194_amd/libkpm.so.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(CSRC, "_build")
LIB = os.path.join(PKG, "libkpm.so")

ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")

# Packed-FP32 instructions are disabled: the compiler then emits scalar FP32 ops only.
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


HEADERS = glob.glob(os.path.join(CSRC, "*.h")) + [os.path.join(ROOT, "include", "kpm.h")]


def _compile(src: str, only_changed: bool = False) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    if only_changed and os.path.exists(obj):
        newest = max(os.path.getmtime(f) for f in [src, *HEADERS])
        if os.path.getmtime(obj) >= newest:
            return obj
    cmd = [HIPCC, *FLAGS, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False, only_changed: bool = False) -> str:
    """Compile every source (only_changed=True: skip objects newer than their
    source and the headers) and link libkpm.so."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(lambda src: _compile(src, only_changed), srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True, only_changed="--changed" in sys.argv)
    sys.exit(0)
