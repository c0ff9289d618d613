"""Scene-level pins for the FP64 oracle: contact sets, surrogate epsilons,
Lemma 1 for the exact descent, and the energy gradient."""
import numpy as np
import pytest

import oracle
import scenegen as sg


@pytest.fixture(scope="module")
def two_spheres_s3():
    s = sg.two_spheres_s3_f64()
    return s, oracle.fine_scene(s)


def test_prereject_never_changes_the_set(two_spheres_s3):
    _, fs = two_spheres_s3
    a = oracle.find_contacts(fs, prereject=True)
    b = oracle.find_contacts(fs, prereject=False)
    assert a["tested"] < b["tested"]
    assert np.array_equal(a["ti"], b["ti"]) and np.array_equal(a["tj"], b["tj"])
    assert np.array_equal(a["d"], b["d"])
    # threshold inclusive: every contact has d <= eps_i + eps_j = 0.1
    assert np.all(a["d"] <= 0.1) and len(a["d"]) > 100


def test_dense_distances_certified(two_spheres_s3):
    """All 1.64M distances of the two-sphere s=3 scene pass the separation
    certificate (or are intersections with coincident points)."""
    s, fs = two_spheres_s3
    r = oracle.find_contacts(fs, delta=np.inf, prereject=False)
    F = len(s.particles[0].fine)
    assert len(r["d"]) == F * F
    A = fs.verts[fs.tris[fs.tri_begin[0] + r["ti"]]]
    B = fs.verts[fs.tris[fs.tri_begin[1] + r["tj"]]]
    d, p1, p2 = r["d"], r["p1"], r["p2"]
    assert np.allclose(np.einsum("nk,nkj->nj", r["w1"], A), p1, atol=1e-12)
    assert np.allclose(np.einsum("nk,nkj->nj", r["w2"], B), p2, atol=1e-12)
    pos = d > 1e-9
    u = (p2[pos] - p1[pos]) / d[pos, None]
    lower = np.einsum("nj,nkj->nk", u, B[pos]).min(1) - np.einsum("nj,nkj->nk", u, A[pos]).max(1)
    assert np.all(lower >= d[pos] - 1e-12 - 1e-13 / d[pos])
    # the minimum over all pairs equals the contact set's minimum
    c = oracle.find_contacts(fs)
    assert np.min(d) == np.min(c["d"])


def _tree_scene():
    return sg.two_spheres(4, [1, 2, 3, 4], "f32", sep=2.03, stream_id=11, name="t")


def test_surrogate_eps_against_sampling():
    s = _tree_scene()
    p = s.particles[0]
    w = s.world(0)
    t = oracle.tree(s)
    n0 = len(p.levels[0])
    fine0 = t.fine_begin[0]
    rng = np.random.default_rng(0)
    for sid in rng.choice(np.arange(fine0), 12, replace=False):
        # fine descendants of sid
        stack, fine = [sid], []
        while stack:
            q = stack.pop()
            if t.child_count[q] == 0:
                fine.append(q)
            else:
                stack.extend(range(t.child_begin[q], t.child_begin[q] + t.child_count[q]))
        verts = np.unique(t.tris[fine].ravel())
        S = t.verts[t.tris[sid]]
        n = 120
        pts = []
        for i in range(n + 1):
            for j in range(n + 1 - i):
                pts.append(S[0] + i / n * (S[1] - S[0]) + j / n * (S[2] - S[0]))
        pts = np.array(pts)
        dmax = max(np.min(np.linalg.norm(pts - t.verts[v], axis=1)) for v in verts)
        h = max(np.linalg.norm(S[a] - S[b]) for a in range(3) for b in range(3))
        dev = t.eps[sid] - p.eps0
        # sampled distance >= true distance >= sampled - step
        assert dev <= dmax + 1e-12 and dmax <= dev + h / n
    assert np.all(t.eps[t.child_count == 0] == p.eps0)
    assert n0 == 80  # coarsest kept level is s=1


def test_lemma1_exact_descent_equals_flat():
    """Lemma 1: with conservative surrogates the descent finds exactly the
    flat contact set (two spheres and a small lattice with mixed depths)."""
    for s in (_tree_scene(), sg.lattice_scene(3, stream_id=12, s_choices=(2, 3))):
        t = oracle.tree(s)
        dsc = oracle.descent(t)
        fs = oracle.fine_scene(s)
        flat = oracle.find_contacts(fs)
        # map descent (global ids) to (pair, local ti, local tj)
        pi, pj = s.pairs[dsc["pair"], 0], s.pairs[dsc["pair"], 1]
        got = set(zip(dsc["pair"].tolist(), (dsc["ti"] - t.fine_begin[pi]).tolist(),
                      (dsc["tj"] - t.fine_begin[pj]).tolist()))
        want = set(zip(flat["pair"].tolist(), flat["ti"].tolist(), flat["tj"].tolist()))
        assert len(want) > 50 and got == want
        assert dsc["tests_per_depth"].sum() < s.n_fine_pairs / 10


def test_lemma1_detects_planted_shrunk_eps():
    """Planting a mistake in the oracle's epsilons (the deviation term halved,
    or dropped) makes the descent lose contacts: the Lemma 1 comparison
    above is sensitive to it."""
    s = _tree_scene()
    t = oracle.tree(s)
    flat = oracle.find_contacts(oracle.fine_scene(s))
    sur = t.child_count > 0
    good = t.eps.copy()
    for f in (0.5, 0.0):
        t.eps[sur] = 0.05 + f * (good[sur] - 0.05)
        dsc = oracle.descent(t)
        assert len(dsc["d"]) < len(flat["d"])


def _energy(fs, k, verts=None):
    if verts is not None:
        fs = oracle.FineScene(verts, fs.tris, fs.tri_begin, fs.tri_count, fs.vert_begin, fs.eps, fs.pairs)
    c = oracle.find_contacts(fs)
    E, g = oracle.energy_grad(fs, c, k)
    return E, g, c


def test_gradient_finite_differences():
    s = sg.two_spheres(2, None, "f64", sep=2.04, stream_id=13, name="fd")
    fs = oracle.fine_scene(s)
    k = 1e4
    E, g, c = _energy(fs, k)
    assert E > 0 and len(c["d"]) > 5
    # vertices of contact pairs, minus those of ambiguous / intersecting pairs
    pi, pj = s.pairs[c["pair"], 0], s.pairs[c["pair"], 1]
    vi = fs.tris[fs.tri_begin[pi] + c["ti"]]
    vj = fs.tris[fs.tri_begin[pj] + c["tj"]]
    bad = c["ambiguous"] | (c["d"] < 1e-9)
    cand = np.setdiff1d(np.unique(np.concatenate([vi.ravel(), vj.ravel()])),
                        np.unique(np.concatenate([vi[bad].ravel(), vj[bad].ravel()])))
    assert len(cand) > 5
    h = 1e-6
    gmax = np.abs(g).max()
    for v in cand[:12]:
        for r in range(3):
            Vp, Vm = fs.verts.copy(), fs.verts.copy()
            Vp[v, r] += h
            Vm[v, r] -= h
            fd = (_energy(fs, k, Vp)[0] - _energy(fs, k, Vm)[0]) / (2 * h)
            assert abs(fd - g[v, r]) <= 1e-6 * gmax, (v, r, fd, g[v, r])


def test_gradient_newton_third_law_and_torque():
    s = sg.two_spheres(3, None, "f64", sep=2.03, stream_id=14, name="n3")
    fs = oracle.fine_scene(s)
    E, g, c = _energy(fs, 1e4)
    assert E > 0
    # translation invariance: total force zero; rotation invariance: total torque zero
    assert np.abs(g.sum(0)).max() <= 1e-9 * np.abs(g).max()
    tau = np.cross(fs.verts, g).sum(0)
    assert np.abs(tau).max() <= 1e-9 * np.abs(g).max() * np.abs(fs.verts).max()
