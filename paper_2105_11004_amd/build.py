"""Builds liblev.so (HIP kernels + C interface) for gfx950, in-tree.

    python -m paper_2105_11004_amd.build      # or build() from Python

Each source is compiled with hipcc (-O3, --offload-arch=gfx950, packed FP32
instructions disabled) in parallel, then linked into
paper_2105_11004_amd/liblev.so.  Always recompiles.
"""

from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys
from pathlib import Path

PKG = Path(__file__).resolve().parent
ROOT = PKG.parent
CSRC = PKG / "csrc"
INCLUDE = ROOT / "include"
BUILD_DIR = PKG / "_build"
LIB = PKG / "liblev.so"
ARCH = "gfx950"

SOURCES = ["sketch.hip", "gauss.hip", "gemm.hip", "pivchol.hip", "rrqr.hip", "trsm.hip", "rownorm.hip",
           "rownorm_bf16.hip", "rownorm_csr.hip", "bwd.hip", "xgemm.hip", "gram_csr.hip", "srht.hip", "qless.hip", "precond.hip",
           "probe.hip", "lev_api.cpp"]

COMMON_FLAGS = [
    "-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
    f"-I{INCLUDE}", f"-I{CSRC}",
]


def _hipcc() -> str:
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not Path(exe).exists():
        raise RuntimeError("hipcc not found; liblev cannot be built")
    return exe


def _compile(src: str) -> Path:
    out = BUILD_DIR / (src + ".o")
    lang = ["-x", "hip"] if src.endswith(".hip") else ["-x", "hip"]
    cmd = [_hipcc(), *lang, "-c", str(CSRC / src), "-o", str(out), *COMMON_FLAGS]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"compiling {src} failed:\n{' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    return out


def build(verbose: bool = False) -> Path:
    BUILD_DIR.mkdir(exist_ok=True)
    jobs = min(len(SOURCES), max(1, min(8, os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB.with_suffix(".so.tmp")
    cmd = [_hipcc(), "-shared", f"--offload-arch={ARCH}", "-o", str(tmp), *map(str, objs)]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"linking liblev failed:\n{' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
