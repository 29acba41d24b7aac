"""Build liblos.so (HIP for gfx950) in-tree.

Every HIP translation unit is compiled with hipcc for gfx950 only, with packed
FP32 VALU instructions disabled (`-Xclang -target-feature -Xclang
-packed-fp32-ops`), then linked into ``paper_2509_25110_amd/liblos.so``.

Run as ``python -m paper_2509_25110_amd.build`` (or via ``__graft_entry__.build``).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "liblos.so")

# heaviest translation units first (the pool compiles them in this order)
SOURCES = ["project_fp64_desc_n3.hip", "project_fp64_desc_n4.hip", "project_fp64_desc_n3s.hip",
           "project_fp64_desc_n4s.hip", "project_fp64_desc_n2.hip", "project_fp64_desc_n2s.hip",
           "project_fp64_desc_n1.hip", "project_fp64_desc_n1s.hip", "project_fp64.hip",
           "emu_kernels.hip", "project_fused.hip", "project_mfma.hip", "project_mfma_lds.hip",
           "spline.hip", "los_api.cpp", "batch_api.cpp", "emu_api.cpp", "bessel_table.hip",
           "project_fp64_desc.hip", "cl_reduce.hip", "jtable.hip", "batch_cl.hip", "cl_interp.hip",
           "tensor.hip", "finite_check.hip"]
# host build of the Bessel seed functions, for CPU checks (not linked into liblos.so)
HOSTCHECK_SRC = "bessel_host_check.cpp"
HOSTCHECK_LIB = os.path.join(PKG, "liblos_hostcheck.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
CFLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wno-unused-result", "-I" + INCLUDE, "-I" + CSRC]


def _headers(src_path, seen=None):
    """Project headers that `src_path` includes, directly or through other project headers."""
    seen = set() if seen is None else seen
    for line in open(src_path):
        line = line.strip()
        if not line.startswith('#include "'):
            continue
        name = line.split('"')[1]
        for d in (CSRC, INCLUDE):
            h = os.path.join(d, name)
            if os.path.exists(h) and h not in seen:
                seen.add(h)
                _headers(h, seen)
                break
    return sorted(seen)


def _compile(src: str, incremental: bool = False) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    if incremental and os.path.exists(obj):
        path = os.path.join(CSRC, src)
        newest = max(os.path.getmtime(p) for p in _headers(path) + [path])
        if os.path.getmtime(obj) > newest:
            return obj
    cmd = [HIPCC, *CFLAGS, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, " ".join(cmd), r.stderr))
    return obj


def build(verbose: bool = True, incremental: bool = False) -> str:
    """Compile all sources and link liblos.so; returns the library path.
    incremental=True reuses objects newer than their source and every header."""
    if shutil.which(HIPCC) is None and not os.path.exists(HIPCC):
        raise RuntimeError("hipcc not found (%s)" % HIPCC)
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(lambda src: _compile(src, incremental), SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH, *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (" ".join(cmd), r.stderr))
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    build_hostcheck(verbose)
    return LIB


def build_hostcheck(verbose: bool = True) -> str:
    """Host-only shared library of the seed functions in bessel_dev.hpp (CPU tests)."""
    tmp = HOSTCHECK_LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, *CFLAGS, "-shared", "-x", "hip", os.path.join(CSRC, HOSTCHECK_SRC), "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (HOSTCHECK_SRC, " ".join(cmd), r.stderr))
    os.replace(tmp, HOSTCHECK_LIB)
    if verbose:
        print("built", HOSTCHECK_LIB)
    return HOSTCHECK_LIB


if __name__ == "__main__":
    build(incremental="--incremental" in sys.argv)
    sys.exit(0)
