"""Builds libgdf.so (HIP, gfx950) in-tree with hipcc.

Every source is compiled to an object under paper_1506_02079_amd/_build/ and
linked into paper_1506_02079_amd/libgdf.so.  Device code is built with packed
FP32 instructions disabled and a high pragma-unroll threshold (the multigrid
and smoothing kernels rely on fully unrolled register rings).
"""
from __future__ import annotations

import os
import re
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libgdf.so")
INCLUDE = os.path.join(ROOT, "include")

SOURCES = ["smooth_rz_b.hip", "mg_kernels.hip", "smooth_rz_d.hip", "smooth_rz_e.hip", "smooth_rz_f.hip",
           "smooth_rz_a.hip", "smooth_rz_c.hip", "tile_kernels.hip", "periodic_kernels.hip", "smooth_kernel.hip",
           "smooth_transpose.hip", "api.cpp"]

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
ARCH = os.environ.get("GDF_OFFLOAD_ARCH", "gfx950")
COMMON = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH, "-I", INCLUDE, "-I", CSRC,
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-mllvm", "-pragma-unroll-threshold=1000000"]


def _deps(path: str, seen: set) -> set:
    """The file and the local headers it includes, transitively."""
    if path in seen or not os.path.exists(path):
        return seen
    seen.add(path)
    for line in open(path):
        m = re.match(r'\s*#\s*include\s+"([^"]+)"', line)
        if m:
            for d in (CSRC, INCLUDE):
                _deps(os.path.join(d, m.group(1)), seen)
    return seen


def _stale(src: str, obj: str) -> bool:
    """The object is older than its source or than a header it includes."""
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(p) > t for p in _deps(os.path.join(CSRC, src), set()))


def _compile(src: str, force: bool = True) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    if not force and not _stale(src, obj):
        return obj
    cmd = [HIPCC] + COMMON + ["-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".cpp"):
        cmd = [HIPCC] + COMMON + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, " ".join(cmd), r.stderr[-8000:]))
    return obj


def build(jobs: int = 8, force: bool = True) -> str:
    """Compile the sources and link libgdf.so; returns the library path.
    force=False recompiles only objects older than their source or a header."""
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=max(1, min(jobs, len(SOURCES)))) as ex:
        objs = list(ex.map(lambda src: _compile(src, force), SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (" ".join(cmd), r.stderr[-8000:]))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    import sys
    print(build(force="--changed" not in sys.argv))
