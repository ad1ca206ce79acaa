"""Build libfca.so (HIP, gfx950) in-tree with hipcc.

Every HIP source is compiled for gfx950 only, with packed-FP32 instruction
selection disabled (-Xclang -target-feature -Xclang -packed-fp32-ops), then
linked into ``paper_1805_06572_amd/libfca.so``. Run ``python -m
paper_1805_06572_amd.build`` or call ``build()``.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OBJ = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libfca.so")
SOURCES = ["fca_conv_m8.hip", "fca_conv_m7.hip", "fca_conv_m6.hip", "fca_conv_m5.hip", "fca_conv_lo.hip",
           "fca_em_nt256.hip", "fca_em_nt128.hip", "fca_kernels.hip", "fca_mlp.hip", "fca_api.hip",
           "fca_noalloc.hip", "fca_stft.hip", "fca_multi.hip"]
ARCH = "gfx950"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def _compile(src: str) -> str:
    obj = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def _deps(path: str, seen: set) -> set:
    """The file and the local headers it includes, recursively."""
    if path in seen or not os.path.exists(path):
        return seen
    seen.add(path)
    for line in open(path):
        line = line.strip()
        if line.startswith('#include "'):
            name = line.split('"')[1]
            for d in (CSRC, os.path.join(ROOT, "include")):
                if os.path.exists(os.path.join(d, name)):
                    _deps(os.path.join(d, name), seen)
    return seen


def _stale(src: str) -> bool:
    obj = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
    if not os.path.exists(obj):
        return True
    deps = _deps(os.path.join(CSRC, src), set())
    return max(os.path.getmtime(d) for d in deps) > os.path.getmtime(obj)


def build(verbose: bool = False, force: bool = True) -> str:
    """Compile the HIP sources and link libfca.so. force=True (the default)
    recompiles everything; force=False only sources newer than their object
    (any header change counts for every source)."""
    os.makedirs(OBJ, exist_ok=True)
    todo = [s for s in SOURCES if force or _stale(s)]
    with ThreadPoolExecutor(max_workers=max(len(todo), 1)) as ex:
        list(ex.map(_compile, todo))
    objs = [os.path.join(OBJ, os.path.splitext(s)[0] + ".o") for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, force="--changed" not in sys.argv)
    sys.exit(0)
