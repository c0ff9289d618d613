"""FP64 CPU oracle for triangle-mesh contact detection (ctypes wrapper).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline use this package; the product path (``paper_2105_12415_amd``) never
imports it.  The arithmetic lives in ``dem_oracle.c`` (plain C, double
precision, no fast-math); this wrapper only converts scenes from
``scenegen`` into the oracle's own array layout and back.

Which passage of the paper each function follows is stated in
``dem_oracle.c``.  Every function here is pinned by tests that do not reuse
its own formulas (closed forms, brute-force sampling, optimality
certificates, finite differences, Lemma 1).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dem_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile dem_oracle.c into liboracle.so (gcc, -O2, no fast-math)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-std=c11",
               "-Wall", "-o", _LIB + ".tmp", _SRC, "-lpthread", "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Contacts(C.Structure):
    _fields_ = [("n", C.c_int64), ("pair", C.POINTER(C.c_int32)), ("ti", C.POINTER(C.c_int32)),
                ("tj", C.POINTER(C.c_int32)), ("rec", C.POINTER(C.c_double)), ("tested", C.c_int64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int32)
        L.oracle_tri_tri.argtypes = [dp, dp, dp]
        L.oracle_set_ambiguity_tol.argtypes = [C.c_double]
        L.oracle_tri_tri_batch.argtypes = [dp, C.c_int64, dp, C.c_int]
        L.oracle_point_triangle.argtypes = [dp, dp, dp]
        L.oracle_segment_segment.argtypes = [dp, dp, dp]
        L.oracle_find_contacts.argtypes = [dp, ip, ip, ip, dp, ip, C.c_int64, C.c_double, C.c_int,
                                           C.c_int, C.POINTER(_Contacts)]
        L.oracle_free_contacts.argtypes = [C.POINTER(_Contacts)]
        L.oracle_energy_grad.argtypes = [ip, C.c_int64, ip, ip, dp, dp, C.c_double, dp, dp]
        L.oracle_surrogate_eps.argtypes = [dp, ip, ip, C.POINTER(C.c_uint8), C.c_int64, C.c_double, dp]
        L.oracle_descent.argtypes = [dp, ip, ip, ip, ip, ip, dp, ip, C.c_int64, C.c_int,
                                     C.POINTER(C.c_int64), C.POINTER(_Contacts)]
        _lib = L
    return _lib


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(C.POINTER(C.c_double))


def _i(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(C.POINTER(C.c_int32))


def set_ambiguity_tol(rel: float = 1e-9) -> None:
    """Candidates within rel * (largest edge) of the minimum, with different
    closest points, mark a pair 'ambiguous' (closest points not unique at
    that resolution).  Process-wide; default 1e-9."""
    lib().oracle_set_ambiguity_tol(float(rel))


def default_threads() -> int:
    return max(1, len(os.sched_getaffinity(0)))


# ----------------------------------------------------------------- primitives
FIELDS = ("d", "p1", "p2", "w1", "w2", "feature", "ambiguous")


def _unpack(rec: np.ndarray) -> dict:
    return {"d": rec[..., 0], "p1": rec[..., 1:4], "p2": rec[..., 4:7], "w1": rec[..., 7:10],
            "w2": rec[..., 10:13], "feature": rec[..., 13].astype(np.int32),
            "ambiguous": rec[..., 14].astype(bool)}


def tri_tri(A, B) -> dict:
    """Exact distance between triangles A, B ((3,3) vertex rows)."""
    A, pa = _d(A)
    B, pb = _d(B)
    out = np.zeros(15)
    lib().oracle_tri_tri(pa, pb, out.ctypes.data_as(C.POINTER(C.c_double)))
    return _unpack(out)


def tri_tri_batch(pairs: np.ndarray, n_threads: int = 0) -> dict:
    """pairs: (n, 2, 3, 3) -> dict of arrays (exact distances etc.)."""
    P, pp = _d(np.asarray(pairs).reshape(-1, 18))
    n = len(P)
    out = np.zeros((n, 15))
    lib().oracle_tri_tri_batch(pp, n, out.ctypes.data_as(C.POINTER(C.c_double)),
                               n_threads or default_threads())
    return _unpack(out)


def point_triangle(p, X) -> dict:
    p, pp = _d(p)
    X, px = _d(X)
    out = np.zeros(7)
    lib().oracle_point_triangle(pp, px, out.ctypes.data_as(C.POINTER(C.c_double)))
    return {"d": out[0], "q": out[1:4], "w": out[4:7]}


def segment_segment(P, Q) -> dict:
    P, pp = _d(P)
    Q, pq = _d(Q)
    out = np.zeros(9)
    lib().oracle_segment_segment(pp, pq, out.ctypes.data_as(C.POINTER(C.c_double)))
    return {"d": out[0], "s": out[1], "t": out[2], "cp": out[3:6], "cq": out[6:9]}


# ----------------------------------------------------------------- scenes
@dataclass
class FineScene:
    """The oracle's own view of a scene: fine triangles only."""
    verts: np.ndarray      # (V,3) f64 world coordinates (rounded to the scene precision)
    tris: np.ndarray       # (T,3) int32 global vertex ids, fine triangles
    tri_begin: np.ndarray  # (P,) first fine triangle of each particle
    tri_count: np.ndarray  # (P,)
    vert_begin: np.ndarray # (P,) first vertex of each particle
    eps: np.ndarray        # (P,) fine-level epsilon
    pairs: np.ndarray      # (n,2) candidate particle pairs


def fine_scene(scene, verts_override=None) -> FineScene:
    """Convert a ``scenegen.Scene``; ``verts_override[p]`` replaces world(p)."""
    vs, ts, tb, tc, vb = [], [], [], [], []
    nv = nt = 0
    for p, part in enumerate(scene.particles):
        w = scene.world(p) if verts_override is None else np.asarray(verts_override[p], np.float64)
        vs.append(w)
        ts.append(part.fine.astype(np.int64) + nv)
        vb.append(nv)
        tb.append(nt)
        tc.append(len(part.fine))
        nv += len(w)
        nt += len(part.fine)
    return FineScene(np.concatenate(vs), np.concatenate(ts).astype(np.int32),
                     np.array(tb, np.int32), np.array(tc, np.int32), np.array(vb, np.int64),
                     np.array([p.eps0 for p in scene.particles]), np.asarray(scene.pairs, np.int32))


def _take(res: _Contacts) -> dict:
    n = res.n
    if n:
        pair = np.ctypeslib.as_array(res.pair, (n,)).copy()
        ti = np.ctypeslib.as_array(res.ti, (n,)).copy()
        tj = np.ctypeslib.as_array(res.tj, (n,)).copy()
        rec = np.ctypeslib.as_array(res.rec, (n, 15)).copy()
    else:
        pair = ti = tj = np.zeros(0, np.int32)
        rec = np.zeros((0, 15))
    out = {"pair": pair, "ti": ti, "tj": tj, "tested": int(res.tested)}
    out.update(_unpack(rec))
    out["rec"] = rec
    lib().oracle_free_contacts(C.byref(res))
    return out


def find_contacts(fs: FineScene, delta: float | None = None, prereject: bool = True,
                  pairs=None, n_threads: int = 0) -> dict:
    """All fine triangle pairs with exact distance <= delta (default eps_i+eps_j).

    ``delta=np.inf`` returns every pair with its exact distance (no rejection).
    ti / tj are particle-local fine triangle indices; output sorted by
    (pair, ti, tj).  ``pairs`` restricts to a subset of candidate pairs (rows
    of fs.pairs); the returned 'pair' indexes that subset.
    """
    V, pv = _d(fs.verts.reshape(-1))
    T, pt = _i(fs.tris.reshape(-1))
    TB, ptb = _i(fs.tri_begin)
    TC, ptc = _i(fs.tri_count)
    E, pe = _d(fs.eps)
    P, pp = _i((fs.pairs if pairs is None else pairs).reshape(-1))
    res = _Contacts()
    lib().oracle_find_contacts(pv, pt, ptb, ptc, pe, pp, len(P) // 2,
                               float("nan") if delta is None else float(delta), int(prereject),
                               n_threads or default_threads(), C.byref(res))
    return _take(res)


def energy_grad(fs: FineScene, contacts: dict, k: float, pairs=None):
    """(E, grad (V,3)) of E = k * sum (delta - d)^2 over the oracle's contacts."""
    P = fs.pairs if pairs is None else pairs
    pi = P[contacts["pair"], 0]
    pj = P[contacts["pair"], 1]
    gti = (fs.tri_begin[pi] + contacts["ti"]).astype(np.int32)
    gtj = (fs.tri_begin[pj] + contacts["tj"]).astype(np.int32)
    delta = fs.eps[pi] + fs.eps[pj]
    T, pt = _i(fs.tris.reshape(-1))
    GI, pgi = _i(gti)
    GJ, pgj = _i(gtj)
    R, pr = _d(contacts["rec"].reshape(-1))
    D, pd = _d(delta)
    grad = np.zeros((len(fs.verts), 3))
    E = np.zeros(1)
    lib().oracle_energy_grad(pt, len(gti), pgi, pgj, pr, pd, float(k),
                             E.ctypes.data_as(C.POINTER(C.c_double)),
                             grad.ctypes.data_as(C.POINTER(C.c_double)))
    return float(E[0]), grad


# ----------------------------------------------------------------- hierarchy
@dataclass
class OracleTree:
    """All-level triangles of a scene in the oracle's numbering."""
    verts: np.ndarray        # (V,3)
    tris: np.ndarray         # (N,3) global vertex ids, particle by particle, coarsest level first
    parent: np.ndarray       # (N,) global parent id or -1
    child_begin: np.ndarray  # (N,)
    child_count: np.ndarray  # (N,) 0 = fine
    eps: np.ndarray          # (N,) oracle surrogate epsilons (eps0 on fine triangles)
    root_begin: np.ndarray   # (P,)
    root_count: np.ndarray   # (P,)
    fine_begin: np.ndarray   # (P,) global id of the first fine triangle
    pairs: np.ndarray


def surrogate_eps(verts: np.ndarray, tris: np.ndarray, parent: np.ndarray, is_fine: np.ndarray,
                  eps0: float) -> np.ndarray:
    V, pv = _d(verts.reshape(-1))
    T, pt = _i(tris.reshape(-1))
    Pa, ppa = _i(parent)
    F = np.ascontiguousarray(is_fine, dtype=np.uint8)
    out = np.zeros(len(parent))
    lib().oracle_surrogate_eps(pv, pt, ppa, F.ctypes.data_as(C.POINTER(C.c_uint8)), len(parent),
                               float(eps0), out.ctypes.data_as(C.POINTER(C.c_double)))
    return out


def tree(scene, verts_override=None) -> OracleTree:
    vs, ts, par, cb, cc, eps, rb, rc, fb = [], [], [], [], [], [], [], [], []
    nv = nt = 0
    for p, part in enumerate(scene.particles):
        w = scene.world(p) if verts_override is None else np.asarray(verts_override[p], np.float64)
        offs = np.cumsum([0] + [len(l) for l in part.levels])
        n = int(offs[-1])
        t_loc = np.concatenate(part.levels).astype(np.int64)
        parent = np.full(n, -1, np.int64)
        cbeg = np.zeros(n, np.int64)
        ccnt = np.zeros(n, np.int64)
        absolute = getattr(part, "parents_absolute", False)
        for l in range(1, len(part.levels)):
            pa = part.parents[l].astype(np.int64) + (0 if absolute else offs[l - 1])
            parent[offs[l]:offs[l + 1]] = pa + nt
            ids = np.arange(offs[l], offs[l + 1])
            # children of one parent are contiguous; parents may sit in any
            # earlier level (particle-local ids in pa)
            first = np.full(offs[l], -1, np.int64)
            for i_loc, pp in zip(ids[::-1], pa[::-1]):
                first[pp] = i_loc
            cnt = np.bincount(pa, minlength=offs[l])
            has = cnt > 0
            cbeg[:offs[l]][has] = first[has] + nt
            ccnt[:offs[l]][has] = cnt[has]
        is_fine = ccnt == 0
        e = surrogate_eps(w, t_loc, np.where(parent >= 0, parent - nt, -1), is_fine, part.eps0)
        vs.append(w)
        ts.append(t_loc + nv)
        par.append(parent)
        cb.append(np.where(ccnt > 0, cbeg, 0))
        cc.append(ccnt)
        eps.append(e)
        rb.append(nt)
        rc.append(len(part.levels[0]))
        fb.append(nt + offs[-2])
        nv += len(w)
        nt += n
    return OracleTree(np.concatenate(vs), np.concatenate(ts).astype(np.int32),
                      np.concatenate(par).astype(np.int32), np.concatenate(cb).astype(np.int32),
                      np.concatenate(cc).astype(np.int32), np.concatenate(eps),
                      np.array(rb, np.int32), np.array(rc, np.int32), np.array(fb, np.int64),
                      np.asarray(scene.pairs, np.int32))


def descent(t: OracleTree, pairs=None, n_threads: int = 0) -> dict:
    """Exact pairwise multiresolution descent; contacts as global triangle ids."""
    V, pv = _d(t.verts.reshape(-1))
    T, pt = _i(t.tris.reshape(-1))
    CB, pcb = _i(t.child_begin)
    CC, pcc = _i(t.child_count)
    RB, prb = _i(t.root_begin)
    RC, prc = _i(t.root_count)
    E, pe = _d(t.eps)
    P, pp = _i((t.pairs if pairs is None else pairs).reshape(-1))
    tests = np.zeros(64, np.int64)
    res = _Contacts()
    lib().oracle_descent(pv, pt, pcb, pcc, prb, prc, pe, pp, len(P) // 2,
                         n_threads or default_threads(),
                         tests.ctypes.data_as(C.POINTER(C.c_int64)), C.byref(res))
    out = _take(res)
    out["tests_per_depth"] = tests
    return out
