"""Pins for the FP64 oracle's triangle-distance primitives.

Nothing here re-types the oracle's formulas: values come from hand-derived
closed forms (tests/golden/closed_forms.json), invariances, an optimality
certificate that is independent of how the closest points were found, and
brute-force sampling of the barycentric parameter space.
"""
import json
import os

import numpy as np
import pytest

import oracle
import scenegen as sg

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")


def _sample_triangle(X, n):
    """Barycentric grid with n subdivisions: points covering X with spacing h/n."""
    pts = []
    for i in range(n + 1):
        for j in range(n + 1 - i):
            a, b = i / n, j / n
            pts.append(X[0] + a * (X[1] - X[0]) + b * (X[2] - X[0]))
    return np.array(pts)


def _diam(X):
    return max(np.linalg.norm(X[i] - X[j]) for i in range(3) for j in range(3))


@pytest.mark.parametrize("case", json.load(open(GOLDEN))["cases"], ids=lambda c: c["name"])
def test_closed_forms(case):
    A, B = np.array(case["A"], float), np.array(case["B"], float)
    r = oracle.tri_tri(A, B)
    assert abs(r["d"] - case["d"]) <= 1e-14 * max(1.0, case["d"])
    # returned points realise the distance and lie on their triangles
    assert abs(np.linalg.norm(r["p2"] - r["p1"]) - r["d"]) <= 1e-14
    assert np.allclose(r["w1"] @ A, r["p1"], atol=1e-14) and np.allclose(r["w2"] @ B, r["p2"], atol=1e-14)
    assert r["w1"].min() >= -1e-15 and r["w2"].min() >= -1e-15
    # swap symmetry (vii)
    s = oracle.tri_tri(B, A)
    assert abs(s["d"] - r["d"]) <= 1e-15
    if not r["ambiguous"]:
        assert np.allclose(s["p1"], r["p2"], atol=1e-13) and np.allclose(s["p2"], r["p1"], atol=1e-13)


def test_vertex_face_gradient():
    """(iv): d/d(vertex) of the distance of a vertex above a face is the face normal."""
    A = np.array([[0, 0, 0], [4, 0, 0], [0, 4, 0]], float)
    B = np.array([[1, 1, 0.7], [1.5, 1, 2], [1, 1.5, 2]], float)
    h = 1e-6
    g = np.zeros(3)
    for k in range(3):
        Bp, Bm = B.copy(), B.copy()
        Bp[0, k] += h
        Bm[0, k] -= h
        g[k] = (oracle.tri_tri(A, Bp)["d"] - oracle.tri_tri(A, Bm)["d"]) / (2 * h)
    assert np.allclose(g, [0, 0, 1], atol=1e-8)


def _certificate(pairs, res, tol, dir_err=1e-15):
    """Separation certificate: along u = (p2-p1)/d every vertex of A lies
    behind p1 and every vertex of B beyond p2, so |p2-p1| equals the
    distance (lower bound u.(p2-p1) = d); for d = 0 the two points coincide
    and lie on their triangles."""
    A, B = pairs[:, 0], pairs[:, 1]
    d, p1, p2, w1, w2 = res["d"], res["p1"], res["p2"], res["w1"], res["w2"]
    # points are convex combinations of the vertices
    assert np.all(w1 >= -1e-12) and np.all(w2 >= -1e-12)
    assert np.allclose(w1.sum(1), 1) and np.allclose(w2.sum(1), 1)
    assert np.allclose(np.einsum("nk,nkj->nj", w1, A), p1, atol=1e-12)
    assert np.allclose(np.einsum("nk,nkj->nj", w2, B), p2, atol=1e-12)
    assert np.allclose(np.linalg.norm(p2 - p1, axis=1), d, atol=1e-13)
    pos = d > 1e-12
    u = (p2[pos] - p1[pos]) / d[pos, None]
    hA = np.einsum("nj,nkj->nk", u, A[pos]).max(1)
    hB = np.einsum("nj,nkj->nk", u, B[pos]).min(1)
    lower = hB - hA
    scale = np.abs(A).max() + np.abs(B).max()
    # the direction u carries the points' rounding error divided by d, which
    # moves the lower bound by that times the triangle extent (dir_err is the
    # relative point error: ~1e-15 in general, larger for nearly parallel
    # edges, whose closest points are ill-conditioned along the edges)
    allow = tol * scale + dir_err * scale * scale / d[pos]
    assert np.all(lower >= d[pos] - allow), np.max(d[pos] - lower - allow)
    return pos


def test_certificate_random_pairs():
    P = sg.random_triangle_pairs(200000, seed=1)
    res = oracle.tri_tri_batch(P)
    pos = _certificate(P, res, 1e-12)
    assert pos.sum() > 100000 and (~pos).sum() > 1000  # both separated and intersecting cases


def test_certificate_near_parallel_and_tiny():
    rng = np.random.default_rng(3)
    n = 50000
    A = rng.uniform(-1, 1, (n, 3, 3))
    # near-parallel copies shifted by a small offset, and tiny triangles
    B = A + rng.normal(0, 1e-3, (n, 3, 3)) + rng.normal(0, 0.05, (n, 1, 3))
    P = np.stack([A, B], 1)
    res = oracle.tri_tri_batch(P)
    _certificate(P, res, 1e-12, dir_err=1e-11)
    # the distance itself is well conditioned: brute force on a subset
    for k in range(0, n, n // 40):
        SA, SB = _sample_triangle(P[k, 0], 30), _sample_triangle(P[k, 1], 30)
        m = np.min(np.linalg.norm(SA[:, None] - SB[None], axis=2))
        assert res["d"][k] - 1e-12 <= m <= res["d"][k] + (_diam(P[k, 0]) + _diam(P[k, 1])) / 30
    T = np.stack([A * 1e-3, A * 1e-3 + rng.normal(0, 1e-3, (n, 1, 3))], 1)
    _certificate(T, oracle.tri_tri_batch(T), 5e-12, dir_err=1e-13)


def test_dense_sampling_bound():
    """Brute force: the sampled minimum is >= d and within the sampling step."""
    P = sg.random_triangle_pairs(60, seed=2)
    res = oracle.tri_tri_batch(P)
    n = 40
    for k in range(len(P)):
        A, B = P[k]
        SA, SB = _sample_triangle(A, n), _sample_triangle(B, n)
        m = np.min(np.linalg.norm(SA[:, None] - SB[None], axis=2))
        d = res["d"][k]
        assert m >= d - 1e-12
        assert m <= d + (_diam(A) + _diam(B)) / n + 1e-12


def degenerate_pairs(n, seed=5):
    """Pairs with a degenerate triangle: collinear vertices (a segment), a
    repeated vertex, all three equal (a point), and a collinear triangle
    against a sliver of relative width 1e-9."""
    rng = np.random.default_rng(seed)
    P = np.zeros((n, 2, 3, 3))
    for i in range(n):
        A = rng.uniform(-1, 1, (3, 3))
        B = rng.uniform(-1, 1, (3, 3)) + rng.uniform(-1.5, 1.5, 3)
        kind = i % 4
        if kind == 0:
            A[2] = A[0] + 0.37 * (A[1] - A[0])
        elif kind == 1:
            A[1] = A[0]
        elif kind == 2:
            A[1] = A[0]
            A[2] = A[0]
        else:
            A[2] = A[0] + 0.37 * (A[1] - A[0])
            B[1] = B[0] + 1e-9 * (B[2] - B[0])
        P[i] = (A, B) if i % 8 < 4 else (B, A)
    return P


def test_degenerate_triangles_sampling():
    """A triangle without interior (segment, point) is met only through its
    boundary: no edge can cross it.  Brute force bounds d from both sides."""
    P = degenerate_pairs(400)
    res = oracle.tri_tri_batch(P)
    n = 40
    for k in range(0, len(P), 4):
        A, B = P[k]
        SA, SB = _sample_triangle(A, n), _sample_triangle(B, n)
        m = np.min(np.linalg.norm(SA[:, None] - SB[None], axis=2))
        d = res["d"][k]
        assert m >= d - 1e-12, (k, d, m)
        assert m <= d + (_diam(A) + _diam(B)) / n + 1e-12, (k, d, m)


def test_degenerate_closed_forms():
    # a collinear "triangle" (a segment) parallel to a face, above its interior
    face = np.array([[0.0, 0.0, 0.0], [2.0, 0.0, 0.0], [0.0, 2.0, 0.0]])
    seg = np.array([[0.2, 0.3, 0.25], [0.8, 0.3, 0.25], [0.5, 0.3, 0.25]])
    r = oracle.tri_tri(seg, face)
    assert abs(r["d"] - 0.25) <= 1e-15 and r["feature"] != 15
    # the segment passing through the face's plane inside it: distance 0
    seg2 = np.array([[0.3, 0.3, -0.5], [0.3, 0.3, 0.5], [0.3, 0.3, 0.0]])
    assert oracle.tri_tri(seg2, face)["d"] <= 1e-15
    # a point: the point-to-triangle distance (nearest point on an edge here)
    pt = np.array([[3.0, -1.0, 0.0]] * 3)
    assert abs(oracle.tri_tri(pt, face)["d"] - np.hypot(1.0, 1.0)) <= 1e-15


def test_point_triangle_and_segments_sampling():
    rng = np.random.default_rng(5)
    for _ in range(200):
        X = rng.uniform(-1, 1, (3, 3))
        p = rng.uniform(-2, 2, 3)
        r = oracle.point_triangle(p, X)
        S = _sample_triangle(X, 60)
        m = np.min(np.linalg.norm(S - p, axis=1))
        assert r["d"] <= m + 1e-12 and m <= r["d"] + _diam(X) / 60 + 1e-12
        assert np.allclose(r["w"] @ X, r["q"])
        P, Q = rng.uniform(-1, 1, (2, 3)), rng.uniform(-1, 1, (2, 3))
        s = oracle.segment_segment(P, Q)
        t = np.linspace(0, 1, 401)
        SP = P[0] + t[:, None] * (P[1] - P[0])
        SQ = Q[0] + t[:, None] * (Q[1] - Q[0])
        m = np.min(np.linalg.norm(SP[:, None] - SQ[None], axis=2))
        assert s["d"] <= m + 1e-12
        assert m <= s["d"] + (np.linalg.norm(P[1] - P[0]) + np.linalg.norm(Q[1] - Q[0])) / 400 + 1e-12


def test_rigid_motion_and_scaling():
    P = sg.random_triangle_pairs(5000, seed=4)
    d0 = oracle.tri_tri_batch(P)["d"]
    rng = np.random.default_rng(11)
    R = sg.random_rotation(rng)
    b = rng.uniform(-10, 10, 3)
    d1 = oracle.tri_tri_batch(P @ R.T + b)["d"]
    assert np.allclose(d1, d0, rtol=1e-13, atol=1e-13 * 12)
    d2 = oracle.tri_tri_batch(P * 3.5)["d"]
    assert np.allclose(d2, 3.5 * d0, rtol=1e-13, atol=1e-14)
    # swapping the two triangles of every pair (vii)
    d3 = oracle.tri_tri_batch(P[:, ::-1])["d"]
    assert np.array_equal(d3 == 0, d0 == 0) and np.allclose(d3, d0, rtol=1e-14, atol=1e-15)


def test_parallel_offset_family():
    """(i) over random triangles: a copy shifted along the normal by h, and a
    rotated (about that normal) copy whose projection still overlaps."""
    rng = np.random.default_rng(8)
    for _ in range(500):
        A = rng.uniform(-1, 1, (3, 3))
        n = np.cross(A[1] - A[0], A[2] - A[0])
        n /= np.linalg.norm(n)
        h = rng.uniform(0.01, 2)
        assert abs(oracle.tri_tri(A, A + h * n)["d"] - h) < 1e-13
        c = A.mean(0)
        th = rng.uniform(0, 2 * np.pi)
        K = np.array([[0, -n[2], n[1]], [n[2], 0, -n[0]], [-n[1], n[0], 0]])
        Rn = np.eye(3) + np.sin(th) * K + (1 - np.cos(th)) * K @ K
        B = (A - c) @ Rn.T * 0.3 + c - h * n
        assert abs(oracle.tri_tri(A, B)["d"] - h) < 1e-13
