"""Contact forces from contact points, with redundant points merged (FP64 oracle).

TEST INFRASTRUCTURE ONLY: the tests use this module; the product path never
imports it.

Follows Section 2:
- the contact point of a fine triangle pair lies on the shortest path between
  the triangles, at the centre of the overlap of the two epsilon-segments,
  and its normal n(c) points from it to the closest point of triangle i;
- one contact point gives the force F(c) = n(c)/|n(c)| K_s (1 - |n(c)|/eps)
  sqrt(1 / (1/M(p_i) + 1/M(p_j))) (a spring over the epsilon-area, K_s =
  1000 in the paper) on p_i and -F(c) on p_j; a particle's force is the sum
  over its contact points, its torque the sum of (x(c) - centre) x force;
- the implementation note on redundant contact points: the points of one
  particle pair that are closer than eps are merged into one average point
  before use.

Readings (the paper leaves them open): "closer than eps" is taken
transitively (single linkage: the merged groups are the connected components
of the "closer than eps" graph of one particle pair's points), with eps =
(eps_i + eps_j) / 2; a merged point carries the mean position and the mean
normal of its group; the force law's eps is eps_i, the radius of the
environment n(c) is measured in (for equal epsilons both readings coincide
with the paper); a contact with n(c) = 0 (intersecting triangles) gives no
force.
"""
from __future__ import annotations

import numpy as np
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components
from scipy.spatial import cKDTree

K_S = 1000.0


def contact_points(fs, contacts: dict, pairs=None):
    """(x, n, pi, pj, eps_i, eps_j) of the oracle's contacts (Section 2, R-9)."""
    P = np.asarray(fs.pairs if pairs is None else pairs).reshape(-1, 2)
    pi = P[contacts["pair"], 0]
    pj = P[contacts["pair"], 1]
    ei, ej = fs.eps[pi], fs.eps[pj]
    p1, p2, d = contacts["p1"], contacts["p2"], contacts["d"]
    lam = np.where(d > 0, (d + ei - ej) / (2 * np.where(d > 0, d, 1.0)), 0.0)
    x = p1 + lam[:, None] * (p2 - p1)
    return x, p1 - x, pi, pj, ei, ej


def merge_groups(x: np.ndarray, pi: np.ndarray, pj: np.ndarray, radius: np.ndarray) -> np.ndarray:
    """Group label of every point: the smallest index of its group, where two
    points of the same particle pair closer than that pair's radius share a
    group, transitively."""
    n = len(x)
    labels = np.arange(n)
    if n == 0:
        return labels
    key = pi.astype(np.int64) * (1 << 32) + pj.astype(np.int64)
    rows, cols = [], []
    for k in np.unique(key):
        idx = np.nonzero(key == k)[0]
        r = float(radius[idx[0]])
        if len(idx) < 2 or r <= 0:
            continue
        pairs = cKDTree(x[idx]).query_pairs(r, output_type="ndarray")
        if len(pairs) == 0:
            continue
        dd = np.linalg.norm(x[idx[pairs[:, 0]]] - x[idx[pairs[:, 1]]], axis=1)
        pairs = pairs[dd < r]
        rows.append(idx[pairs[:, 0]])
        cols.append(idx[pairs[:, 1]])
    if rows:
        r_, c_ = np.concatenate(rows), np.concatenate(cols)
        g = coo_matrix((np.ones(len(r_)), (r_, c_)), shape=(n, n))
        _, comp = connected_components(g, directed=False)
        first = np.full(comp.max() + 1, n)
        np.minimum.at(first, comp, np.arange(n))
        labels = first[comp]
    return labels


def force_of(nvec: np.ndarray, eps_i: np.ndarray, mi: np.ndarray, mj: np.ndarray, k_s: float = K_S):
    """F(c) on particle i for normals n(c) (rows)."""
    ln = np.linalg.norm(nvec, axis=1)
    u = np.where(ln[:, None] > 0, nvec / np.where(ln > 0, ln, 1.0)[:, None], 0.0)
    mag = k_s * (1.0 - ln / eps_i) * np.sqrt(1.0 / (1.0 / mi + 1.0 / mj))
    return u * mag[:, None]


def contact_forces(fs, contacts: dict, mass: np.ndarray, centre: np.ndarray, k_s: float = K_S,
                   merge: bool = True, pairs=None) -> dict:
    """Merged contact points, their forces, and per-particle force and torque.

    mass (P,), centre (P,3).  Returns labels (group of every input contact),
    and per group (rows ordered by label): x, n, f (on p_i), pi, pj,
    members; force (P,3) and torque (P,3)."""
    x, nv, pi, pj, ei, ej = contact_points(fs, contacts, pairs)
    labels = merge_groups(x, pi, pj, 0.5 * (ei + ej)) if merge else np.arange(len(x))
    roots, inv, cnt = np.unique(labels, return_inverse=True, return_counts=True)
    G = len(roots)
    xm = np.zeros((G, 3))
    nm = np.zeros((G, 3))
    np.add.at(xm, inv, x)
    np.add.at(nm, inv, nv)
    xm /= np.maximum(cnt, 1)[:, None]
    nm /= np.maximum(cnt, 1)[:, None]
    gpi, gpj = pi[roots], pj[roots]
    f = force_of(nm, ei[roots], mass[gpi], mass[gpj], k_s)
    Pn = len(mass)
    force = np.zeros((Pn, 3))
    torque = np.zeros((Pn, 3))
    np.add.at(force, gpi, f)
    np.add.at(force, gpj, -f)
    np.add.at(torque, gpi, np.cross(xm - centre[gpi], f))
    np.add.at(torque, gpj, np.cross(xm - centre[gpj], -f))
    return {"labels": labels, "x": xm, "n": nm, "f": f, "pi": gpi, "pj": gpj, "members": cnt,
            "force": force, "torque": torque}
