"""Seeded synthetic scenes for multiresolution triangle-mesh contact detection.

This module only *generates inputs*: icosphere meshes and their nesting, radial
bumps, random rigid poses, particle placement, and candidate particle pairs (the
broad phase, which the paper leaves outside the method, Section 6).  It holds
none of the contact method's arithmetic -- no triangle distances, no surrogate
epsilons, no iterations -- so that the FP64 oracle and the HIP path can both
consume it without sharing any of that arithmetic.

The workloads stand in for the paper's "sphere-like" particles (Section 6.1):
the paper perturbs spheres with Perlin noise; here each vertex radius is
perturbed by an i.i.d. uniform bump, which keeps the surfaces closed and
star-shaped around the particle centre.  All randomness comes from
``numpy.random.SeedSequence`` children, so every scene is reproducible.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

SEED = 210512415          # base entropy for every scene
BUMP = 0.05               # absolute radial bump amplitude U(-BUMP, BUMP)
EPS0 = 0.05               # epsilon of every fine triangle (delta = 0.1 per fine pair)


# --------------------------------------------------------------------------- meshes
def _icosahedron():
    """12 unit vertices, 20 outward-oriented faces (sorted, deterministic)."""
    phi = (1.0 + 5.0 ** 0.5) / 2.0
    v = []
    for a in (-1.0, 1.0):
        for b in (-phi, phi):
            v += [(0.0, a, b), (a, b, 0.0), (b, 0.0, a)]
    v = np.array(v, dtype=np.float64)
    n = len(v)
    d = np.linalg.norm(v[:, None, :] - v[None, :, :], axis=2)
    adj = np.abs(d - 2.0) < 1e-9
    faces = []
    for i in range(n):
        for j in range(i + 1, n):
            if not adj[i, j]:
                continue
            for k in range(j + 1, n):
                if adj[i, k] and adj[j, k]:
                    a, b, c = v[i], v[j], v[k]
                    if np.dot(np.cross(b - a, c - a), a + b + c) < 0:
                        faces.append((i, k, j))
                    else:
                        faces.append((i, j, k))
    faces = np.array(faces, dtype=np.int64)
    assert faces.shape == (20, 3)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v, faces


def _subdivide(verts: np.ndarray, faces: np.ndarray):
    """Split every face into 4; children of face f are 4f..4f+3.

    Child 0..2 keep one corner of the parent, child 3 is the centre triangle.
    Edge midpoints are pushed onto the unit sphere and shared between the two
    faces of an edge (new vertices are numbered by sorted edge key).
    """
    F = len(faces)
    V = len(verts)
    a, b, c = faces[:, 0], faces[:, 1], faces[:, 2]
    e = np.concatenate([np.stack([a, b], 1), np.stack([b, c], 1), np.stack([c, a], 1)])
    es = np.sort(e, axis=1)
    key = es[:, 0] * (V + 1) + es[:, 1]
    uniq, first, inv = np.unique(key, return_index=True, return_inverse=True)
    mid = verts[es[first, 0]] + verts[es[first, 1]]
    mid /= np.linalg.norm(mid, axis=1, keepdims=True)
    new_idx = V + np.arange(len(uniq))
    m_ab = new_idx[inv[0:F]]
    m_bc = new_idx[inv[F:2 * F]]
    m_ca = new_idx[inv[2 * F:3 * F]]
    ch = np.empty((F, 4, 3), dtype=np.int64)
    ch[:, 0] = np.stack([a, m_ab, m_ca], 1)
    ch[:, 1] = np.stack([m_ab, b, m_bc], 1)
    ch[:, 2] = np.stack([m_ca, m_bc, c], 1)
    ch[:, 3] = np.stack([m_ab, m_bc, m_ca], 1)
    return np.concatenate([verts, mid]), ch.reshape(4 * F, 3)


_ICO_CACHE: dict = {}


def icosphere(s_max: int):
    """Unit icosphere: (dirs (V,3) f64, [faces_s (20*4^s,3) for s=0..s_max]).

    Vertex numbering is nested: the vertices of level s are the first
    10*4^s+2 entries, so a coarser level's faces index the same array.
    """
    if s_max in _ICO_CACHE:
        v, fl = _ICO_CACHE[s_max]
        return v.copy(), [f.copy() for f in fl]
    v, f = _icosahedron()
    fl = [f]
    for _ in range(s_max):
        v, f = _subdivide(v, f)
        fl.append(f)
    _ICO_CACHE[s_max] = (v, fl)
    return v.copy(), [x.copy() for x in fl]


def random_rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniform random rotation (normalised Gaussian quaternion)."""
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


# --------------------------------------------------------------------------- data
@dataclass
class Particle:
    """One rigid particle: a closed triangulated surface plus its nesting.

    ``levels[0]`` is the coarsest triangle set and ``levels[-1]`` the particle
    triangulation itself.  ``parents[l]`` (l >= 1) gives, for each face of
    level l, the index of the face of level l-1 it was split from; children of
    one parent are contiguous.  For a single-level particle there is no nesting.
    """
    body: np.ndarray                 # (V,3) f64 body-frame vertices (centre at origin)
    rot: np.ndarray                  # (3,3) rotation body -> world
    centre: np.ndarray               # (3,)  translation body -> world
    levels: List[np.ndarray]         # faces per level, local vertex ids, int32
    parents: List[Optional[np.ndarray]]
    radius: float                    # nominal radius R
    subdiv: List[int]                # icosphere subdivision of each level
    eps0: float = EPS0
    parents_absolute: bool = False   # parents[l] index all of the particle's triangles, not level l-1

    @property
    def n_verts(self) -> int:
        return len(self.body)

    @property
    def fine(self) -> np.ndarray:
        return self.levels[-1]

    def world(self, dtype=np.float64) -> np.ndarray:
        """World-frame vertices rounded to ``dtype`` and returned as f64."""
        w = self.body @ self.rot.T + self.centre
        return w.astype(dtype).astype(np.float64)


@dataclass
class Scene:
    name: str
    particles: List[Particle]
    pairs: np.ndarray                # (P,2) int32 candidate particle pairs, i < j
    dtype: str                       # 'f32' or 'f64' arithmetic of the GPU path
    info: dict = field(default_factory=dict)

    @property
    def np_dtype(self):
        return np.float32 if self.dtype == "f32" else np.float64

    def world(self, p: int) -> np.ndarray:
        return self.particles[p].world(self.np_dtype)

    @property
    def n_fine_pairs(self) -> int:
        F = np.array([len(p.fine) for p in self.particles], dtype=np.int64)
        return int(np.sum(F[self.pairs[:, 0]] * F[self.pairs[:, 1]]))


def _streams(stream_id: int, n: int):
    ss = np.random.SeedSequence(SEED, spawn_key=(stream_id,))
    return [np.random.default_rng(c) for c in ss.spawn(n)]


def bumped_sphere(rng: np.random.Generator, s_fine: int, R: float,
                  levels: Optional[Sequence[int]] = None, centre=(0.0, 0.0, 0.0),
                  rotate: bool = True, bump: float = BUMP, eps0: float = EPS0) -> Particle:
    """Icosphere of subdivision ``s_fine`` with radii R + U(-bump, bump).

    ``levels`` lists the subdivisions kept in the hierarchy (ascending, last
    one == s_fine); default: only the fine level.  Random numbers are drawn in
    the order: vertex bumps, then the rotation quaternion.
    """
    levels = [s_fine] if levels is None else list(levels)
    assert levels == sorted(levels) and levels[-1] == s_fine
    dirs, faces = icosphere(s_fine)
    r = R + rng.uniform(-bump, bump, size=len(dirs))
    body = dirs * r[:, None]
    rot = random_rotation(rng) if rotate else np.eye(3)
    lv = [faces[s].astype(np.int32) for s in levels]
    parents: List[Optional[np.ndarray]] = [None]
    for k in range(1, len(levels)):
        ratio = 4 ** (levels[k] - levels[k - 1])
        parents.append((np.arange(len(lv[k])) // ratio).astype(np.int32))
    return Particle(body=body, rot=rot, centre=np.asarray(centre, np.float64), levels=lv,
                    parents=parents, radius=float(R), subdiv=levels, eps0=eps0)


def candidate_pairs(centres: np.ndarray, radii: np.ndarray, margin: float) -> np.ndarray:
    """Particle pairs whose bounding spheres (radius + margin/2 each) overlap."""
    c = np.asarray(centres)
    r = np.asarray(radii)
    out = []
    n = len(c)
    for i in range(n):
        d = np.linalg.norm(c[i + 1:] - c[i], axis=1)
        j = np.nonzero(d <= r[i] + r[i + 1:] + margin)[0] + i + 1
        out.extend((i, int(k)) for k in j)
    return np.array(out, dtype=np.int32).reshape(-1, 2)


def _pair_margin(bump=BUMP, eps0=EPS0) -> float:
    # surfaces lie within R +- bump; contact needs surface distance <= 2 eps0
    return 2.0 * bump + 2.0 * eps0 + 1e-9


# --------------------------------------------------------------------------- workloads
def two_spheres(s_fine: int, levels: Optional[Sequence[int]] = None, dtype: str = "f64",
                sep: float = 2.02, stream_id: int = 1, name: str = "two_spheres") -> Scene:
    """Two bumped unit spheres with centres ``sep`` apart along x."""
    rngs = _streams(stream_id, 2)
    ps = [bumped_sphere(rngs[0], s_fine, 1.0, levels, centre=(0.0, 0.0, 0.0)),
          bumped_sphere(rngs[1], s_fine, 1.0, levels, centre=(sep, 0.0, 0.0))]
    return Scene(name, ps, np.array([[0, 1]], np.int32), dtype,
                 info={"s": s_fine, "levels": list(levels or [s_fine]), "sep": sep})


def two_spheres_s3_f64() -> Scene:
    """Two s=3 bumped unit spheres (1280 tris each), FP64, flat all-pairs."""
    return two_spheres(3, None, "f64", 2.02, 1, "two_spheres_s3_f64_flat")


def two_spheres_s5_hier() -> Scene:
    """Two s=5 bumped unit spheres (20480 tris each), FP32, levels s=3/4/5."""
    return two_spheres(5, [3, 4, 5], "f32", 2.02, 2, "two_spheres_s5_f32_hier345")


def _drop_lattice(R: np.ndarray, rng: np.random.Generator, n: int):
    """Centres for an n^3 lattice of spheres packed with surface gaps U(0, 0.1).

    Rows along x are chains: consecutive spheres are R_a + R_b + g apart.  Each
    sphere is then "dropped" along -y onto the spheres of the earlier rows of
    its plane, and afterwards along -z onto the spheres of the earlier planes:
    it rests on the first sphere it would touch, at its own gap g.  Moving a
    sphere away from others along an axis never creates an overlap, so the
    packing has no overlaps and every sphere has a near neighbour along each
    axis.
    """
    N = n ** 3
    lat = np.stack(np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij"), -1).reshape(-1, 3)
    gx, gy, gz = (rng.uniform(0.0, 0.1, size=N) for _ in range(3))
    c = np.zeros((N, 3))
    id_of = {tuple(t): k for k, t in enumerate(lat)}
    # x chains
    for j in range(n):
        for k in range(n):
            x = 0.0
            for i in range(n):
                a = id_of[(i, j, k)]
                if i > 0:
                    b = id_of[(i - 1, j, k)]
                    x = c[b, 0] + R[a] + R[b] + gx[a]
                c[a, 0] = x

    def drop(a, others, axis, gap):
        if len(others) == 0:
            return None
        keep = [q for q in range(3) if q != axis]
        d2 = np.sum((c[others][:, keep] - c[a, keep]) ** 2, axis=1)
        need = (R[a] + R[others] + gap) ** 2
        hit = d2 < need
        if not np.any(hit):
            return None
        return float(np.max(c[others[hit], axis] + np.sqrt(need[hit] - d2[hit])))

    for k in range(n):
        for j in range(n):
            for i in range(n):
                a = id_of[(i, j, k)]
                if j > 0:
                    prev = np.array([id_of[(ii, jj, k)] for jj in range(j) for ii in range(n)])
                    y = drop(a, prev, 1, gy[a])
                    c[a, 1] = y if y is not None else c[id_of[(i, j - 1, k)], 1]
    for k in range(1, n):
        prev = np.array([id_of[(ii, jj, kk)] for kk in range(k) for jj in range(n) for ii in range(n)])
        for j in range(n):
            for i in range(n):
                a = id_of[(i, j, k)]
                z = drop(a, prev, 2, gz[a])
                c[a, 2] = z if z is not None else c[id_of[(i, j, k - 1)], 2]
    return c


def lattice_scene(n: int = 10, stream_id: int = 3, s_choices=(3, 4, 5),
                  r_range=(0.5, 2.0), name: str = "lattice") -> Scene:
    """n^3 bumped spheres: s ~ U(s_choices), R ~ logU(r_range), lattice gaps U(0,0.1).

    Every particle keeps the whole icosphere cascade s = 0..s_p as its hierarchy.
    """
    N = n ** 3
    rngs = _streams(stream_id, N + 1)
    g_rng = rngs[N]
    s = g_rng.choice(np.asarray(s_choices), size=N)
    R = np.exp(g_rng.uniform(np.log(r_range[0]), np.log(r_range[1]), size=N))
    centres = _drop_lattice(R, g_rng, n)
    D = np.linalg.norm(centres[:, None, :] - centres[None, :, :], axis=2) - R[:, None] - R[None, :]
    np.fill_diagonal(D, np.inf)
    ps = [bumped_sphere(rngs[i], int(s[i]), float(R[i]), list(range(int(s[i]) + 1)),
                        centre=centres[i]) for i in range(N)]
    pairs = candidate_pairs(centres, R + BUMP, 2.0 * EPS0 + 1e-9)
    return Scene(name, ps, pairs, "f32",
                 info={"n": n, "min_nominal_gap": float(D.min()),
                       "pairs_nominal_gap_le_0.1": int(np.sum(np.triu(D <= 0.1, 1))),
                       "subdiv_hist": np.bincount(s, minlength=6).tolist()})


def lattice1000() -> Scene:
    """1000 bumped spheres on a 10^3 lattice, s in {3,4,5}, R logU[0.5,2], FP32."""
    return lattice_scene(10, 3, name="lattice1000_s345_f32")


def _cone_descend(dirs_big: np.ndarray, faces: List[np.ndarray], u: np.ndarray) -> np.ndarray:
    """Index of the finest icosphere face whose cone contains each direction u."""
    def inside(fc, uu):
        a, b, c = dirs_big[fc[:, 0]], dirs_big[fc[:, 1]], dirs_big[fc[:, 2]]
        s1 = np.einsum("ij,ij->i", np.cross(a, b), uu)
        s2 = np.einsum("ij,ij->i", np.cross(b, c), uu)
        s3 = np.einsum("ij,ij->i", np.cross(c, a), uu)
        return np.minimum(np.minimum(s1, s2), s3)
    m = len(u)
    score0 = np.stack([inside(np.repeat(faces[0][k:k + 1], m, 0), u) for k in range(20)], 1)
    f = np.argmax(score0, axis=1)
    for s in range(1, len(faces)):
        cand = 4 * f[:, None] + np.arange(4)[None, :]
        sc = np.stack([inside(faces[s][cand[:, k]], u) for k in range(4)], 1)
        f = cand[np.arange(m), np.argmax(sc, axis=1)]
    return f


def size_disparate_scene(s_big: int = 7, R_big: float = 20.0, n_small: int = 2000,
                         s_small: int = 3, R_small: float = 0.5, gap=(-0.01, 0.05),
                         stream_id: int = 4, name: str = "big_plus_small") -> Scene:
    """One big bumped sphere plus ``n_small`` small ones resting on its surface."""
    rngs = _streams(stream_id, n_small + 2)
    big = bumped_sphere(rngs[0], s_big, R_big, list(range(s_big + 1)), centre=(0, 0, 0))
    g_rng = rngs[1]
    k = np.arange(n_small) + 0.5
    golden = np.pi * (3.0 - 5.0 ** 0.5)
    z = 1.0 - 2.0 * k / n_small
    rr = np.sqrt(1.0 - z * z)
    u = np.stack([rr * np.cos(golden * k), rr * np.sin(golden * k), z], 1)
    spacing = np.sqrt(4.0 * np.pi / n_small)  # on the unit sphere
    u = u + g_rng.uniform(-0.2, 0.2, size=u.shape) * spacing
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    # radius of the bumped big mesh along u (body frame of the big sphere)
    ub = u @ big.rot  # world -> body
    dirs, faces = icosphere(s_big)
    f = _cone_descend(dirs, faces[:s_big + 1], ub)
    tri = faces[s_big][f]
    A, B, C = big.body[tri[:, 0]], big.body[tri[:, 1]], big.body[tri[:, 2]]
    nrm = np.cross(B - A, C - A)
    r_big = np.einsum("ij,ij->i", nrm, A) / np.einsum("ij,ij->i", nrm, ub)
    g = g_rng.uniform(gap[0], gap[1], size=n_small)
    centres = u * (r_big + R_small + g)[:, None]
    smalls = [bumped_sphere(rngs[2 + i], s_small, R_small, list(range(s_small + 1)),
                            centre=centres[i]) for i in range(n_small)]
    ps = [big] + smalls
    allc = np.concatenate([np.zeros((1, 3)), centres])
    allr = np.concatenate([[R_big], np.full(n_small, R_small)]) + BUMP
    pairs = candidate_pairs(allc, allr, 2.0 * EPS0 + 1e-9)
    n_big_small = int(np.sum(pairs[:, 0] == 0))
    return Scene(name, ps, pairs, "f32",
                 info={"n_big_small": n_big_small, "n_small_small": int(len(pairs) - n_big_small)})


def big_plus_small() -> Scene:
    """R=20 s=7 sphere (327680 tris) + 2000 R=0.5 s=3 spheres on it, FP32."""
    return size_disparate_scene(name="big_s7_plus_2000_small_s3_f32")


# --------------------------------------------------------------------------- generic meshes
def bumped_torus(rng: np.random.Generator, nu: int, nv: int, R: float, r: float, bump: float = BUMP):
    """A torus around the z axis (tube radius r + U(-bump, bump) per vertex),
    triangulated from an nu x nv parameter grid with outward orientation: a
    closed mesh with no nesting, for surrogate trees built from scratch.
    Returns (verts (nu*nv, 3) f64, tris (2*nu*nv, 3) int32)."""
    u = 2 * np.pi * np.arange(nu) / nu
    v = 2 * np.pi * np.arange(nv) / nv
    U, Vv = np.meshgrid(u, v, indexing="ij")
    rr = r + rng.uniform(-bump, bump, size=U.shape)
    X = (R + rr * np.cos(Vv)) * np.cos(U)
    Y = (R + rr * np.cos(Vv)) * np.sin(U)
    Z = rr * np.sin(Vv)
    verts = np.stack([X, Y, Z], -1).reshape(-1, 3)
    idx = lambda i, j: (i % nu) * nv + (j % nv)
    tris = []
    for i in range(nu):
        for j in range(nv):
            a, b, c, d = idx(i, j), idx(i + 1, j), idx(i + 1, j + 1), idx(i, j + 1)
            tris += [(a, b, c), (a, c, d)]
    return verts, np.array(tris, np.int32)


def two_tori(nu: int = 48, nv: int = 24, R: float = 1.0, r: float = 0.35, gap: float = 0.02,
             stream_id: int = 6):
    """Two bumped tori side by side along x, rims ``gap`` apart before the
    bumps, each with a random rotation about its own axis; meshes only.
    Returns [(verts, tris, rot, centre), ...]."""
    rngs = _streams(stream_id, 2)
    out = []
    for k in range(2):
        verts, tris = bumped_torus(rngs[k], nu, nv, R, r)
        ang = rngs[k].uniform(0, 2 * np.pi)
        rot = np.array([[np.cos(ang), -np.sin(ang), 0], [np.sin(ang), np.cos(ang), 0], [0, 0, 1.0]])
        centre = np.array([k * (2 * (R + r) + gap), 0.0, 0.0])
        out.append((verts, tris, rot, centre))
    return out


# --------------------------------------------------------------------------- motion
def rigid_perturbations(n_particles: int, n_steps: int, stream_id: int = 5,
                        max_shift: float = 2e-3, max_angle: float = 2e-3):
    """Seeded per-step, per-particle small rigid motions (axis-angle, shift).

    Returns (rotations (n_steps, P, 3, 3), shifts (n_steps, P, 3)) about each
    particle's centre.  Step 0 is the identity.
    """
    rng = _streams(stream_id, 1)[0]
    Rs = np.zeros((n_steps, n_particles, 3, 3))
    ts = np.zeros((n_steps, n_particles, 3))
    for st in range(n_steps):
        if st == 0:
            Rs[st] = np.eye(3)
            continue
        ax = rng.normal(size=(n_particles, 3))
        ax /= np.linalg.norm(ax, axis=1, keepdims=True)
        ang = rng.uniform(0, max_angle, size=n_particles)
        K = np.zeros((n_particles, 3, 3))
        K[:, 0, 1], K[:, 0, 2], K[:, 1, 2] = -ax[:, 2], ax[:, 1], -ax[:, 0]
        K[:, 1, 0], K[:, 2, 0], K[:, 2, 1] = ax[:, 2], -ax[:, 1], ax[:, 0]
        s, c = np.sin(ang)[:, None, None], np.cos(ang)[:, None, None]
        Rs[st] = np.eye(3)[None] + s * K + (1 - c) * (K @ K)
        sh = rng.normal(size=(n_particles, 3))
        sh /= np.linalg.norm(sh, axis=1, keepdims=True)
        ts[st] = sh * rng.uniform(0, max_shift, size=(n_particles, 1))
    return Rs, ts


def random_triangle_pairs(n: int, seed: int = 7, scale: float = 1.0, spread: float = 1.5,
                          dtype=np.float64) -> np.ndarray:
    """(n, 2, 3, 3) random triangle pairs: vertices U(-scale, scale) around two
    centres U(-spread, spread) apart (a mix of separated and intersecting)."""
    rng = np.random.default_rng(np.random.SeedSequence(SEED, spawn_key=(100, seed)))
    c = rng.uniform(-spread, spread, size=(n, 2, 1, 3))
    v = c + rng.uniform(-scale, scale, size=(n, 2, 3, 3))
    return v.astype(dtype).astype(np.float64)


__all__ = [
    "Particle", "Scene", "icosphere", "bumped_sphere", "two_spheres", "two_spheres_s3_f64", "two_spheres_s5_hier",
    "lattice1000", "big_plus_small", "lattice_scene", "size_disparate_scene", "candidate_pairs",
    "rigid_perturbations", "random_rotation", "random_triangle_pairs", "EPS0", "BUMP", "SEED",
]
