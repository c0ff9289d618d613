"""Build libdem.so (HIP for gfx950) in-tree with hipcc.

    python -m paper_2105_12415_amd.build

Packed-FP32 instructions are disabled for every HIP translation unit.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libdem.so")
SOURCES = ["dem_kernels.hip", "dem_hierarchy.cpp", "dem_surrogate.cpp"]
# achievable-peak microbenchmarks (FMA loop, device copy) used by bench.py
PEAK_LIB = os.path.join(HERE, "libpeak.so")
PEAK_SOURCES = ["peak_probe.hip"]
ARCH = os.environ.get("DEM_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for c in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.exists(c) or c == "hipcc":
            return c
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False, lib_path: str = LIB, extra_flags=(), sources=None) -> str:
    """Compile SOURCES (or ``sources``: paths) into ``lib_path``."""
    objs = []
    common = ["-O3", "-std=c++17", "-fPIC", "-I", INCLUDE, "-I", CSRC, "-Wall", "-Wno-unused-function"]
    common += list(extra_flags)
    out_dir = os.path.dirname(os.path.abspath(lib_path))
    for src in (sources or [os.path.join(CSRC, s) for s in SOURCES]):
        path = src
        obj = os.path.join(out_dir, "_obj_" + os.path.splitext(os.path.basename(src))[0] + ".o")
        cmd = [hipcc(), "-c", "-x", "hip", f"--offload-arch={ARCH}",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-munsafe-fp-atomics"] + common + ["-o", obj, path]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = lib_path + ".tmp"
    cmd = [hipcc(), "-shared", f"--offload-arch={ARCH}", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, lib_path)
    for o in objs:
        os.remove(o)
    return lib_path


def build_all(verbose: bool = False):
    """libdem.so and libpeak.so."""
    build(verbose)
    build(verbose, lib_path=PEAK_LIB, sources=[os.path.join(CSRC, s) for s in PEAK_SOURCES])


if __name__ == "__main__":
    build_all(verbose="-v" in sys.argv)
    print(LIB, PEAK_LIB)
