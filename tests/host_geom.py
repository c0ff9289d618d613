"""Host build of the product's triangle geometry, for CPU tests only."""
import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc", "geom_host.cpp")
LIB = os.path.join(HERE, "csrc", "libgeom_host.so")
_lib = None


def lib():
    global _lib
    if _lib is None:
        hdr = os.path.join(ROOT, "paper_2105_12415_amd", "csrc", "dem_geom.hpp")
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < max(os.path.getmtime(SRC), os.path.getmtime(hdr)):
            subprocess.check_call(["/opt/rocm/bin/hipcc", "-x", "hip", "--offload-arch=gfx950", "-O2",
                                   "-ffp-contract=off", "-shared", "-fPIC", "-std=c++17",
                                   "-I", os.path.join(ROOT, "paper_2105_12415_amd", "csrc"),
                                   "-o", LIB + ".tmp", SRC])
            os.replace(LIB + ".tmp", LIB)
        L = C.CDLL(LIB)
        dp = C.POINTER(C.c_double)
        L.geom_exact.argtypes = [dp, C.c_long, C.c_int, dp]
        L.geom_bound.argtypes = [dp, C.c_long, C.c_int, C.POINTER(C.c_float), dp]
        L.geom_certify.argtypes = [dp, C.c_long, C.c_int, C.POINTER(C.c_float), dp]
        _lib = L
    return _lib


def exact(pairs, double=True):
    P = np.ascontiguousarray(np.asarray(pairs, np.float64).reshape(-1, 18))
    out = np.zeros((len(P), 14))
    lib().geom_exact(P.ctypes.data_as(C.POINTER(C.c_double)), len(P), int(double),
                     out.ctypes.data_as(C.POINTER(C.c_double)))
    return {"d": out[:, 0], "p1": out[:, 1:4], "p2": out[:, 4:7], "w1": out[:, 7:10],
            "w2": out[:, 10:13], "feature": out[:, 13].astype(int)}


def bound(pairs, double=True, n_iter=4, omega=1.0, areg=1e-4, rho=1e3, centroid=0, half=False):
    """half: the reduced-precision iteration (FP32 only)."""
    P = np.ascontiguousarray(np.asarray(pairs, np.float64).reshape(-1, 18))
    prm = np.array([n_iter, omega, areg, rho, centroid, 1.0 if half else 0.0], np.float32)
    out = np.zeros((len(P), 7))
    lib().geom_bound(P.ctypes.data_as(C.POINTER(C.c_double)), len(P), int(double),
                     prm.ctypes.data_as(C.POINTER(C.c_float)), out.ctypes.data_as(C.POINTER(C.c_double)))
    return {"L": out[:, 0], "slack": out[:, 1], "up": out[:, 2], "theta": out[:, 3:7]}


def certify(pairs, double=True, omega=1.0, areg=1e-4, rho=1e3, centroid=0):
    P = np.ascontiguousarray(np.asarray(pairs, np.float64).reshape(-1, 18))
    prm = np.array([4, omega, areg, rho, centroid, 0.0], np.float32)
    out = np.zeros((len(P), 2))
    lib().geom_certify(P.ctypes.data_as(C.POINTER(C.c_double)), len(P), int(double),
                       prm.ctypes.data_as(C.POINTER(C.c_float)), out.ctypes.data_as(C.POINTER(C.c_double)))
    return {"ok": out[:, 0] > 0, "d": out[:, 1]}
