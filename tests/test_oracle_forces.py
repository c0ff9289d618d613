"""Pins of the oracle's contact forces and merging (Section 2: force of a
contact point, equal and opposite on the two particles; implementation note
on redundant contact points merged when closer than eps)."""
from types import SimpleNamespace

import numpy as np

import oracle
import scenegen as sg
from oracle import forces as of

SQRT_6_5 = 1.0954451150103321  # sqrt(1 / (1/2 + 1/3)) for masses 2 and 3


def _one_contact(eps_i, eps_j, d):
    fs = SimpleNamespace(eps=np.array([eps_i, eps_j]), pairs=np.array([[0, 1]]))
    c = {"pair": np.array([0]), "p1": np.array([[0.0, 0.0, 0.0]]), "p2": np.array([[0.0, 0.0, -d]]),
         "d": np.array([d])}
    return fs, c


def test_single_contact_force_closed_form():
    fs, c = _one_contact(0.05, 0.05, 0.06)
    r = of.contact_forces(fs, c, np.array([2.0, 3.0]), np.zeros((2, 3)))
    # x halfway, n = (0, 0, 0.03): K_s (1 - 0.03/0.05) sqrt(6/5) along +z on particle 0
    assert np.allclose(r["x"], [[0, 0, -0.03]], atol=1e-15)
    assert np.allclose(r["f"], [[0, 0, 400.0 * SQRT_6_5]], rtol=1e-14)
    assert np.allclose(r["force"], [[0, 0, 400.0 * SQRT_6_5], [0, 0, -400.0 * SQRT_6_5]], rtol=1e-14)
    # unequal environments: x at the centre of the overlap [d - eps_j, eps_i] = [0, 0.04] from p1
    fs, c = _one_contact(0.04, 0.06, 0.06)
    r = of.contact_forces(fs, c, np.array([2.0, 3.0]), np.zeros((2, 3)))
    assert np.allclose(r["x"], [[0, 0, -0.02]], atol=1e-15)
    assert np.allclose(r["f"], [[0, 0, 500.0 * SQRT_6_5]], rtol=1e-14)
    # intersecting triangles: no direction, no force
    fs, c = _one_contact(0.05, 0.05, 0.0)
    r = of.contact_forces(fs, c, np.array([2.0, 3.0]), np.zeros((2, 3)))
    assert np.all(r["f"] == 0)


def test_torque_closed_form():
    fs, c = _one_contact(0.05, 0.05, 0.06)
    centre = np.array([[1.0, 0.0, 0.0], [0.0, 2.0, 0.0]])
    r = of.contact_forces(fs, c, np.array([2.0, 3.0]), centre)
    F = 400.0 * SQRT_6_5
    # (x - c0) x (0,0,F) with x - c0 = (-1, 0, -0.03): (0*F - (-0.03)*0, -0.03*0 - (-1)*F, 0) = (0, F, 0)
    assert np.allclose(r["torque"][0], [0, F, 0], rtol=1e-14)
    # (x - c1) x (0,0,-F) with x - c1 = (0, -2, -0.03): (-2*-F - 0, 0 - 0, 0) = (2F, 0, 0)
    assert np.allclose(r["torque"][1], [2 * F, 0, 0], rtol=1e-14)


def test_merge_is_single_linkage_within_a_pair():
    r = 0.05
    x = np.array([[0, 0, 0], [0.9 * r, 0, 0], [1.8 * r, 0, 0],      # chain: one group
                  [5, 0, 0], [5 + 1.1 * r, 0, 0],                  # too far: two groups
                  [0, 0, 0]], dtype=float)                         # same place, other pair
    pi = np.array([0, 0, 0, 0, 0, 0])
    pj = np.array([1, 1, 1, 1, 1, 2])
    lab = of.merge_groups(x, pi, pj, np.full(6, r))
    assert lab.tolist() == [0, 0, 0, 3, 4, 5]


def test_vertex_to_vertex_duplicates_merge_into_one_point():
    """The implementation note's example: two particles whose closest points
    are two vertices; every pair of triangles around them reports the same
    contact point, and merging leaves one."""
    rng = np.random.default_rng(0)
    a = sg.bumped_sphere(rng, 0, 1.0, bump=0.0, rotate=False)
    b = sg.bumped_sphere(rng, 0, 1.0, bump=0.0, rotate=False)
    v = a.body[0] / np.linalg.norm(a.body[0])
    b.centre = (2.0 + 0.05) * v  # b's vertex -v faces a's vertex v, 0.05 apart
    sc = sg.Scene("vv", [a, b], np.array([[0, 1]], np.int32), "f64")
    fs = oracle.fine_scene(sc)
    c = oracle.find_contacts(fs)
    assert len(c["d"]) == 25 and np.allclose(c["d"], 0.05, atol=1e-12)
    r = of.contact_forces(fs, c, np.array([1.0, 1.0]), np.zeros((2, 3)))
    assert len(r["f"]) == 1 and r["members"][0] == 25
    # n = 0.025 v: K_s (1 - 0.5) sqrt(1/2) along -v... on particle 0, pushing it away from particle 1
    assert np.allclose(r["f"][0], -500.0 * np.sqrt(0.5) * v, rtol=1e-9, atol=1e-9)
    unmerged = of.contact_forces(fs, c, np.array([1.0, 1.0]), np.zeros((2, 3)), merge=False)
    assert len(unmerged["f"]) == 25 and np.allclose(unmerged["force"], 25 * r["force"], rtol=1e-9)


def test_third_law_and_angular_momentum_on_spheres():
    sc = sg.two_spheres_s3_f64()
    fs = oracle.fine_scene(sc)
    c = oracle.find_contacts(fs)
    mass = np.array([1.0, 1.7])
    centre = np.array([p.centre for p in sc.particles])
    for merge in (True, False):
        r = of.contact_forces(fs, c, mass, centre, merge=merge)
        assert len(r["f"]) > 0
        scale = np.abs(r["force"]).max()
        assert np.allclose(r["force"].sum(0), 0, atol=1e-12 * scale)
        L = r["torque"] + np.cross(centre, r["force"])
        assert np.allclose(L.sum(0), 0, atol=1e-12 * scale)
    merged = of.contact_forces(fs, c, mass, centre, merge=True)
    assert len(merged["f"]) < len(c["d"])
    # a merged point lies in the bounding box of its group
    x, *_ = of.contact_points(fs, c)
    for g, root in enumerate(np.unique(merged["labels"])):
        m = x[merged["labels"] == root]
        assert np.all(merged["x"][g] >= m.min(0) - 1e-12) and np.all(merged["x"][g] <= m.max(0) + 1e-12)


def test_merge_groups_match_brute_force_single_linkage():
    """merge_groups (k-d tree pairs + connected components) against a
    brute-force single linkage written out directly: all pairwise distances,
    a union-find over the pairs closer than the radius, within one particle
    pair only; labels are the smallest index of each group."""
    rng = np.random.default_rng(11)
    n = 400
    x = rng.uniform(0, 1, (n, 3)) * np.array([1.0, 1.0, 0.2])
    pi = rng.integers(0, 3, n)
    pj = pi + 1 + rng.integers(0, 2, n)
    radius = np.where(pi == 0, 0.06, 0.09)
    lab = of.merge_groups(x, pi, pj, radius)
    parent = list(range(n))

    def find(a):
        while parent[a] != a:
            a = parent[a]
        return a
    for a in range(n):
        for b in range(a + 1, n):
            if pi[a] == pi[b] and pj[a] == pj[b] and np.sqrt(((x[a] - x[b]) ** 2).sum()) < radius[a]:
                ra, rb = find(a), find(b)
                if ra != rb:
                    parent[max(ra, rb)] = min(ra, rb)
    want = np.array([find(a) for a in range(n)])
    assert np.array_equal(lab, want)
    assert len(np.unique(want)) < n  # some points did merge
