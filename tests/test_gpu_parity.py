"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Bars (written in each test): distances |d_gpu - d_ref| <= r d_ref + a h
(h = longest edge of the pair; FP32 r=1e-5 a=1e-6, FP64 r=1e-12 a=1e-13);
contact sets identical except pairs within the threshold band (FP32 1e-6,
FP64 1e-12) of delta = eps_i + eps_j; gradients per vertex within 1e-4
(FP32) of the largest oracle gradient, vertices of pairs whose
closest points are not unique at that resolution excluded; the summed
FP64 gradient within 1e-10 of the largest oracle gradient.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
import scenegen as sg
from paper_2105_12415_amd import _abi, api

pytestmark = pytest.mark.gpu

TOL = {"f32": dict(r=1e-5, a=1e-6, band=1e-6, g=1e-4, amb=1e-5),
       "f64": dict(r=1e-12, a=1e-13, band=1e-12, g=1e-10, amb=1e-9)}


def say(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(autouse=True)
def _announce(request):
    say(f"[gpu-test] {request.node.nodeid}")
    yield
    oracle.set_ambiguity_tol()


def run(scene, mode="hier", **kw):
    ds = api.DeviceScene(scene, device="cuda:0")
    eng = api.ContactEngine(ds, api.make_params(mode, **kw))
    status = eng.run()
    assert status == 0, hex(status)
    return ds, eng, eng.result()


def keyed(ds, res):
    """(pi, pj, local ti, local tj) -> index, for GPU results."""
    lti = res["ti"] - ds.fine_begin_host[res["pi"]]
    ltj = res["tj"] - ds.fine_begin_host[res["pj"]]
    return {(int(a), int(b), int(c), int(d)): k for k, (a, b, c, d) in
            enumerate(zip(res["pi"], res["pj"], lti, ltj))}


def oracle_keyed(scene, ref):
    P = np.asarray(scene.pairs)
    return {(int(P[p, 0]), int(P[p, 1]), int(a), int(b)): k for k, (p, a, b) in
            enumerate(zip(ref["pair"], ref["ti"], ref["tj"]))}


def pair_geom(fs, pi, pj, ti, tj):
    A = fs.verts[fs.tris[fs.tri_begin[pi] + ti]]
    B = fs.verts[fs.tris[fs.tri_begin[pj] + tj]]
    return A, B


def longest_edge(A, B):
    e = [np.linalg.norm(X[(k + 1) % 3] - X[k]) for X in (A, B) for k in range(3)]
    return max(e)


def compare_sets(scene, ds, res, ref, tol, fs=None):
    fs = fs or oracle.fine_scene(scene)
    g = keyed(ds, res)
    o = oracle_keyed(scene, ref)
    delta = 2 * scene.particles[0].eps0
    only_gpu = set(g) - set(o)
    only_ref = set(o) - set(g)
    for key in only_ref:
        d = ref["d"][o[key]]
        assert abs(d - delta) <= tol["band"], ("missed contact", key, d)
    for key in only_gpu:
        A, B = pair_geom(fs, *key)
        d = oracle.tri_tri(A, B)["d"]
        assert abs(d - delta) <= tol["band"], ("spurious contact", key, d)
    common = sorted(set(g) & set(o))
    dg = np.array([res["d"][g[k]] for k in common])
    dr = np.array([ref["d"][o[k]] for k in common])
    h = np.array([longest_edge(*pair_geom(fs, *k)) for k in common]) if len(common) < 200000 else 1.0
    err = np.abs(dg - dr) - (tol["r"] * dr + tol["a"] * h)
    assert np.all(err <= 0), (np.max(err), common[int(np.argmax(err))])
    return len(common), len(only_gpu), len(only_ref)


# ------------------------------------------------------------------ distances
def test_dense_fp64_all_distances_two_spheres_s3():
    """1,638,400 exact FP64 distances (flat, threshold +inf) vs the oracle."""
    scene = sg.two_spheres_s3_f64()
    ds, eng, res = run(scene, "flat", dense_distance=1)
    F = len(scene.particles[0].fine)
    assert len(res["d"]) == F * F
    fs = oracle.fine_scene(scene)
    ref = oracle.find_contacts(fs, delta=np.inf, prereject=False)
    lti = res["ti"] - ds.fine_begin_host[0]
    ltj = res["tj"] - ds.fine_begin_host[1]
    order = np.lexsort((ltj, lti))
    assert np.array_equal(lti[order], ref["ti"]) and np.array_equal(ltj[order], ref["tj"])
    dg = res["d"][order]
    A = fs.verts[fs.tris[fs.tri_begin[0] + ref["ti"]]]
    B = fs.verts[fs.tris[fs.tri_begin[1] + ref["tj"]]]
    h = np.maximum(np.linalg.norm(A - np.roll(A, 1, 1), axis=2).max(1),
                   np.linalg.norm(B - np.roll(B, 1, 1), axis=2).max(1))
    err = np.abs(dg - ref["d"]) - (1e-12 * ref["d"] + 1e-13 * h)
    assert np.all(err <= 0), np.max(err)


@pytest.mark.parametrize("mode", ["flat", "hier"])
def test_contacts_fp64_two_spheres_s3(mode):
    scene = sg.two_spheres_s3_f64()
    ds, eng, res = run(scene, mode)
    ref = oracle.find_contacts(oracle.fine_scene(scene))
    n, og, orf = compare_sets(scene, ds, res, ref, TOL["f64"])
    assert n > 100
    E_ref, _ = oracle.energy_grad(oracle.fine_scene(scene), ref, 1e4)
    assert abs(res["energy"] - E_ref) <= 1e-10 * E_ref


@pytest.mark.parametrize("mode", ["flat", "hier"])
def test_contacts_fp32_two_spheres_s4_levels(mode):
    scene = sg.two_spheres(4, [1, 2, 3, 4], "f32", sep=2.03, stream_id=41, name="s4")
    ds, eng, res = run(scene, mode)
    ref = oracle.find_contacts(oracle.fine_scene(scene))
    n, og, orf = compare_sets(scene, ds, res, ref, TOL["f32"])
    assert n > 500
    E_ref, _ = oracle.energy_grad(oracle.fine_scene(scene), ref, 1e4)
    assert abs(res["energy"] - E_ref) <= 1e-5 * E_ref
    if mode == "hier":
        st = eng.stats_dict()
        # the descent evaluates far fewer pairs than all fine pairs
        assert st["evals"].sum() < ds.n_fine_pairs() / 20


def test_hier_equals_flat_and_oracle_config2():
    """Two s=5 spheres (20480 tris each), levels s=3/4/5, FP32: Lemma 1."""
    scene = sg.two_spheres_s5_hier()
    ds, eng, res_h = run(scene, "hier")
    _, eng_f, res_f = run(scene, "flat")
    ref = oracle.find_contacts(oracle.fine_scene(scene))
    compare_sets(scene, ds, res_h, ref, TOL["f32"])
    compare_sets(scene, ds, res_f, ref, TOL["f32"])
    kh, kf = keyed(ds, res_h), keyed(ds, res_f)
    assert set(kh) == set(kf)  # same FP32 arithmetic on the fine pairs
    # GPU descent tests at least as many pairs as an exact descent
    t = oracle.tree(scene)
    dsc = oracle.descent(t)
    st = eng.stats_dict()
    assert st["evals"].sum() >= dsc["tests_per_depth"].sum()


def test_lattice_mixed_depths():
    """27 spheres with s in {2,3} and radii 0.5-2: uneven depths per pair."""
    scene = sg.lattice_scene(3, stream_id=42, s_choices=(2, 3))
    ds, eng, res = run(scene, "hier")
    ref = oracle.find_contacts(oracle.fine_scene(scene))
    n, og, orf = compare_sets(scene, ds, res, ref, TOL["f32"])
    assert n > 100


def _lazy_eager_run(scene, lazy, dense):
    ds = api.DeviceScene(scene, device="cuda:0", lazy=lazy)
    assert ds.lazy == lazy and (ds.c.fine_parents is not None) == lazy
    P = ds.n_particles
    Rs, ts = sg.rigid_perturbations(P, 3)
    centres = np.array([p.centre for p in scene.particles])
    shift = centres + ts[2] - np.einsum("pij,pj->pi", Rs[2], centres)
    pose = np.concatenate([Rs[2].reshape(P, 9), shift], 1)
    ds.set_pose(torch.as_tensor(pose, dtype=ds.dtype, device="cuda:0").contiguous())
    eng = api.ContactEngine(ds, api.make_params("hier", dense_distance=dense), energy_k=1e4,
                            contact_capacity=1 << 20)
    assert eng.run() == 0
    res = eng.result()
    grad = torch.zeros(3, ds.n_verts, dtype=ds.dtype, device="cuda:0")
    eng.backward(grad, energy=True)
    torch.cuda.synchronize()
    assert eng.check() == 0
    order = np.lexsort((res["tj"], res["ti"]))
    return ({k: np.asarray(res[k])[order] for k in ("ti", "tj", "d")}, float(eng.energy_bwd.item()),
            grad.cpu().numpy())


@pytest.mark.parametrize("case", ["lattice_depths_2_4", "two_spheres_dense"])
def test_lazy_flatten_matches_eager(case):
    """Lazy flattening (fine records written only below surviving surrogates)
    against writing every record: identical contacts and distances, bit for
    bit, and the same energy and gradient up to the order of atomic sums, on
    an uneven-depth scene moved by per-particle poses, and in dense-distance
    mode (every fine pair reported, so every fine record is needed)."""
    if case == "lattice_depths_2_4":
        scene, dense, n_min = sg.lattice_scene(3, stream_id=44, s_choices=(2, 3, 4)), 0, 100
    else:
        scene = sg.two_spheres(2, [0, 1, 2], "f32", sep=2.03, stream_id=45, name="dense")
        dense, n_min = 1, 320 * 320
    ra, ea, ga = _lazy_eager_run(scene, True, dense)
    rb, eb, gb = _lazy_eager_run(scene, False, dense)
    assert len(ra["d"]) >= n_min
    for k in ("ti", "tj", "d"):
        assert np.array_equal(ra[k], rb[k]), k
    assert abs(ea - eb) <= 1e-12 * abs(eb) + 1e-300
    assert np.allclose(ga, gb, rtol=1e-5, atol=1e-6 * np.abs(gb).max())


def _degenerate_scene(dtype):
    """Two s=2 spheres (levels 0..2) whose facing sides carry degenerate fine
    triangles: a vertex collapsed onto its neighbour (a repeated vertex) and
    a vertex moved to the middle of an opposite edge (collinear vertices)."""
    scene = sg.two_spheres(2, [0, 1, 2], dtype, sep=2.03, stream_id=46, name="degenerate")
    for p, sign in ((0, 1.0), (1, -1.0)):
        part = scene.particles[p]
        w = part.body @ part.rot.T
        tris = part.fine
        facing = np.argsort(-sign * w[tris].mean(1)[:, 0])[:12]  # faces towards the other sphere
        for n, f in enumerate(facing[::2]):
            i, j, k = tris[f]
            if n % 2 == 0:
                part.body[j] = part.body[i]
            else:
                part.body[k] = 0.5 * (part.body[i] + part.body[j])
    return scene


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_degenerate_triangles_scene(prec):
    """Segments and repeated vertices among the fine triangles: every fine
    pair's exact distance (dense mode) and the hierarchical contact set
    against the oracle."""
    scene = _degenerate_scene(prec)
    fs = oracle.fine_scene(scene)
    tris = fs.tris
    A = fs.verts[tris]
    area2 = np.linalg.norm(np.cross(A[:, 1] - A[:, 0], A[:, 2] - A[:, 0]), axis=1)
    assert np.sum(area2 <= 1e-12 * np.max(area2)) >= 6  # the scene really holds degenerate triangles
    ds, eng, res = run(scene, "hier", dense_distance=1)
    ref = oracle.find_contacts(fs, delta=np.inf, prereject=False)
    g = keyed(ds, res)
    o = oracle_keyed(scene, ref)
    assert set(g) == set(o)
    common = sorted(o)
    dg = np.array([res["d"][g[k]] for k in common])
    dr = np.array([ref["d"][o[k]] for k in common])
    h = np.array([longest_edge(*pair_geom(fs, *k)) for k in common])
    tol = TOL[prec]
    err = np.abs(dg - dr) - (tol["r"] * dr + tol["a"] * h)
    assert np.all(err <= 0), (np.max(err), common[int(np.argmax(err))])
    ds, eng, res = run(scene, "hier")
    n, _, _ = compare_sets(scene, ds, res, oracle.find_contacts(fs), tol, fs)
    assert n > 10


@pytest.mark.parametrize("mode", ["hier", "flat"])
@pytest.mark.parametrize("case", ["no_pairs", "far_apart"])
def test_empty_inputs(mode, case):
    """No candidate pairs, or a pair whose particles are too far apart for any
    contact: no contacts, zero energy, zero gradient, clean status."""
    scene = sg.two_spheres(2, [0, 1, 2], "f32", sep=2.03 if case == "no_pairs" else 3.0,
                           stream_id=47, name=case)
    if case == "no_pairs":
        scene.pairs = np.zeros((0, 2), np.int32)
    ds = api.DeviceScene(scene, device="cuda:0")
    eng = api.ContactEngine(ds, api.make_params(mode), energy_k=1e4)
    assert eng.run() == 0
    res = eng.result()
    assert len(res["d"]) == 0 and res["energy"] == 0.0
    grad = torch.ones(3, ds.n_verts, dtype=ds.dtype, device="cuda:0")
    eng.backward(grad, energy=True)
    torch.cuda.synchronize()
    assert eng.check() == 0
    assert float(eng.energy_bwd.item()) == 0.0
    assert bool(torch.all(grad == 1.0))  # accumulated into, nothing added
    if case == "far_apart":
        assert oracle.find_contacts(oracle.fine_scene(scene))["d"].size == 0


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_generic_mesh_surrogate_trees(prec):
    """Two bumped tori (a parametric mesh, no nesting) with surrogate trees
    from the library's k-means builder: leaf sets at different depths, fine
    triangles below surrogates of several levels.  Hierarchical contacts
    against the oracle and against the flat path."""
    from generic_mesh import two_tori_scene
    scene, _ = two_tori_scene(prec)
    fs = oracle.fine_scene(scene)
    ref = oracle.find_contacts(fs)
    ds, eng, res = run(scene, "hier")
    assert ds.n_levels_max >= 4 and ds.lazy
    n, _, _ = compare_sets(scene, ds, res, ref, TOL[prec], fs)
    assert n > 100
    _, _, flat = run(scene, "flat")
    assert set(keyed(ds, flat)) == set(keyed(ds, res))


# ------------------------------------------------------------------ gradients
def _grad_compare(scene, prec):
    tol = TOL[prec]
    ds = api.DeviceScene(scene, device="cuda:0")
    eng = api.ContactEngine(ds, api.make_params("hier"), energy_k=1e4)
    verts = ds.verts.clone().requires_grad_(True)
    E = api.contact_energy(verts, eng)
    assert eng.check() == 0
    E.backward()
    torch.cuda.synchronize()
    g = verts.grad.double().cpu().numpy().T
    fs = oracle.fine_scene(scene)
    oracle.set_ambiguity_tol(tol["amb"])
    ref = oracle.find_contacts(fs)
    E_ref, g_ref = oracle.energy_grad(fs, ref, 1e4)
    assert abs(float(E.detach()) - E_ref) <= (1e-5 if prec == "f32" else 1e-10) * E_ref
    # exclude vertices of pairs with non-unique closest points at this
    # resolution, and of pairs within the threshold band (in or out)
    P = np.asarray(scene.pairs)
    bad = ref["ambiguous"] | (np.abs(ref["d"] - 0.1) <= tol["band"])
    vi = fs.tris[fs.tri_begin[P[ref["pair"], 0]] + ref["ti"]]
    vj = fs.tris[fs.tri_begin[P[ref["pair"], 1]] + ref["tj"]]
    skip = np.unique(np.concatenate([vi[bad].ravel(), vj[bad].ravel()]))
    keep = np.ones(len(g), bool)
    keep[skip] = False
    gmax = np.abs(g_ref).max()
    err = np.abs(g - g_ref)[keep].max() / gmax
    assert err <= tol["g"], err
    assert keep.sum() > 0.9 * len(np.unique(np.concatenate([vi.ravel(), vj.ravel()])))


def test_gradient_fp64():
    _grad_compare(sg.two_spheres(3, [1, 2, 3], "f64", sep=2.03, stream_id=43, name="g64"), "f64")


def test_gradient_fp32():
    _grad_compare(sg.two_spheres(4, [2, 3, 4], "f32", sep=2.03, stream_id=44, name="g32"), "f32")


def test_adjoint_central_differences_fp64():
    """dem_contact_backward against central finite differences of the GPU's
    own FP64 energy (dem_find_contacts), on two small spheres: step h = 1e-6
    on single world coordinates, two coordinates of each of the 40 vertices
    with the largest gradients.  E is C^1 across the threshold and has no
    jumps, so with closest points that are unique (oracle ambiguity flag),
    pairs off the band and not intersecting, the difference quotient is
    within O(h^2) (third derivative) + O(u E / h) (rounding) of dE/dv: the
    bar is 1e-6 of the largest gradient, per coordinate."""
    scene = sg.two_spheres(3, [1, 2, 3], "f64", sep=2.03, stream_id=43, name="fd64")
    ds = api.DeviceScene(scene, device="cuda:0")
    eng = api.ContactEngine(ds, api.make_params("hier"), energy_k=1e4)
    assert eng.run() == 0
    grad = torch.zeros(3, ds.n_verts, dtype=ds.dtype, device="cuda:0")
    eng.backward(grad)
    torch.cuda.synchronize()
    g = grad.cpu().numpy().T.copy()
    fs = oracle.fine_scene(scene)
    oracle.set_ambiguity_tol(1e-6)
    ref = oracle.find_contacts(fs)
    P = np.asarray(scene.pairs)
    # vertices whose pairs could switch features or cross d = 0 within a step
    bad = ref["ambiguous"] | (ref["d"] < 1e-4) | (np.abs(ref["d"] - 0.1) <= 1e-4)
    vi = fs.tris[fs.tri_begin[P[ref["pair"], 0]] + ref["ti"]]
    vj = fs.tris[fs.tri_begin[P[ref["pair"], 1]] + ref["tj"]]
    skip = np.unique(np.concatenate([vi[bad].ravel(), vj[bad].ravel()]))
    cand = np.setdiff1d(np.unique(np.concatenate([vi.ravel(), vj.ravel()])), skip)
    assert len(cand) > 40
    gmax = np.abs(g).max()
    pick = cand[np.argsort(-np.abs(g[cand]).max(1))[:40]]
    h = 1e-6
    verts = ds.verts
    worst = 0.0
    for v in pick:
        for c in (int(np.argmax(np.abs(g[v]))), int(np.argmin(np.abs(g[v])))):
            x0 = float(verts[c, v])
            e = []
            for sgn in (1.0, -1.0):
                verts[c, v] = x0 + sgn * h
                eng.forward()
                assert eng.check() == 0
                e.append(float(eng.energy.item()))
            verts[c, v] = x0
            fd = (e[0] - e[1]) / (2 * h)
            worst = max(worst, abs(fd - g[v, c]) / gmax)
            assert abs(fd - g[v, c]) <= 1e-6 * gmax, (int(v), c, fd, g[v, c])
    say(f"[gpu-test] central differences: {2 * len(pick)} coordinates, worst {worst:.2e} of max |g|")


# ------------------------------------------------------------------ forced failures
def _fine_only_vertex(scene, p):
    """A vertex of particle p that only fine triangles use (not a vertex of
    any coarser level)."""
    part = scene.particles[p]
    coarse = np.unique(np.concatenate(part.levels[:-1]))
    only = np.setdiff1d(np.unique(part.fine), coarse)
    assert len(only)
    return int(only[0])


@pytest.mark.parametrize("where", ["root_vertex", "fine_only_vertex_pruned"])
def test_nonfinite_vertex_sets_status(where):
    """A NaN coordinate is ordinary input: the call completes, sets
    DEM_DEV_NONFINITE, and run() raises.  In lazy mode a fine-only vertex
    below surrogates that are all pruned (spheres far apart) is never read
    by a soup record, and is still reported."""
    sep = 2.03 if where == "root_vertex" else 3.0
    scene = sg.two_spheres(3, [0, 1, 2, 3], "f32", sep=sep, stream_id=51, name="nan")
    ds = api.DeviceScene(scene, device="cuda:0")
    assert ds.lazy
    v = 0 if where == "root_vertex" else _fine_only_vertex(scene, 1)
    v_global = int(ds.vert_begin[1]) + v
    ds.verts[1, v_global] = float("nan")
    eng = api.ContactEngine(ds, api.make_params("hier"), energy_k=1e4)
    eng.forward()
    status = eng.check()
    say(f"[gpu-test] NaN at {where}: status {status:#x}, {eng.count()} contacts")
    assert status & _abi.DEM_DEV_NONFINITE
    if where != "root_vertex":
        assert eng.count() == 0  # nothing else changed
    with pytest.raises(api.DemError):
        eng.run()


@pytest.mark.parametrize("certify", [0, 1])
def test_no_regulariser_same_contacts(certify):
    """alpha_reg -> 0 (1e-30 of the edge lengths): the iteration's Hessian
    loses its regularisation and settles fewer pairs, the exact fallback
    takes the rest, and the contact set and distances are unchanged."""
    scene = sg.two_spheres(3, [1, 2, 3], "f32", sep=2.03, stream_id=46, name="areg")
    ds, e_ref, r_ref = run(scene, "hier")
    _, e0, r0 = run(scene, "hier", alpha_reg_rel=1e-30, certify=certify)
    ref = oracle.find_contacts(oracle.fine_scene(scene))
    n, _, _ = compare_sets(scene, ds, r0, ref, TOL["f32"])
    assert n > 100
    a = sorted(zip(r_ref["ti"].tolist(), r_ref["tj"].tolist(), r_ref["d"].tolist()))
    b = sorted(zip(r0["ti"].tolist(), r0["tj"].tolist(), r0["d"].tolist()))
    if not certify:
        assert a == b  # the same exact distances of the same pairs
    st = e0.stats_dict()
    say(f"[gpu-test] alpha_reg 1e-30, certify={certify}: near {st['near']} (default "
        f"{e_ref.stats_dict()['near']}), certified {st['certified']}")


@pytest.mark.parametrize("which", ["queue", "near"])
def test_overflow_retry_same_contacts(which):
    """A level queue or the near list far too small: the first call reports
    the overflow; run() grows the list from the device counters and repeats
    the call, and the contacts equal those of a call with room to spare."""
    scene = sg.two_spheres(4, [0, 1, 2, 3, 4], "f32", sep=2.02, stream_id=52, name="retry")
    ds, e_ref, r_ref = run(scene, "hier")
    cap = "queue_capacity" if which == "queue" else "near_capacity"
    flag = _abi.DEM_DEV_QUEUE_OVERFLOW if which == "queue" else _abi.DEM_DEV_NEAR_OVERFLOW
    eng = api.ContactEngine(ds, api.make_params("hier", **{cap: 64}))
    eng.forward()
    status = eng.check()
    assert status & flag, hex(status)
    assert eng.run() == 0
    res = eng.result()
    assert getattr(eng.p, cap) > 64
    a = sorted(zip(r_ref["ti"].tolist(), r_ref["tj"].tolist(), r_ref["d"].tolist()))
    b = sorted(zip(res["ti"].tolist(), res["tj"].tolist(), res["d"].tolist()))
    assert len(a) > 100 and a == b


def test_backward_skips_contacts_outside_the_scene():
    """A contact naming a triangle id beyond the scene is skipped by the
    adjoint and reported (DEM_DEV_BAD_TREE); the others still count."""
    scene = sg.two_spheres(3, [1, 2, 3], "f32", sep=2.03, stream_id=46, name="badid")
    ds = api.DeviceScene(scene, device="cuda:0")
    eng = api.ContactEngine(ds, api.make_params("hier"), energy_k=1e4)
    assert eng.run() == 0
    n = eng.count()
    full = eng.contacts
    g0 = torch.zeros(3, ds.n_verts, dtype=ds.dtype, device="cuda:0")
    eng.backward(g0, energy=True)
    torch.cuda.synchronize()
    e0 = float(eng.energy_bwd.item())
    ti = torch.cat([full.ti[:n], torch.tensor([ds.n_tris + 5, -3], dtype=torch.int32, device="cuda:0")])
    tj = torch.cat([full.tj[:n], torch.tensor([0, ds.n_tris], dtype=torch.int32, device="cuda:0")])
    eng.contacts = _sub_contacts(full, ti, tj)
    eng.status.zero_()
    g1 = torch.zeros_like(g0)
    try:
        eng.backward(g1, energy=True)
        torch.cuda.synchronize()
    finally:
        eng.contacts = full
    assert eng.check() & _abi.DEM_DEV_BAD_TREE
    assert abs(float(eng.energy_bwd.item()) - e0) <= 1e-5 * e0
    assert torch.allclose(g1, g0, rtol=1e-5, atol=1e-6 * float(g0.abs().max()))


def test_autograd_backward_after_another_forward_raises():
    """The autograd function's backward differentiates the contacts of its
    own forward; after another forward on the same engine it refuses."""
    scene = sg.two_spheres(3, [1, 2, 3], "f32", sep=2.03, stream_id=46, name="gen")
    ds = api.DeviceScene(scene, device="cuda:0")
    eng = api.ContactEngine(ds, api.make_params("hier"), energy_k=1e4)
    v = ds.verts.clone().requires_grad_(True)
    E = api.contact_energy(v, eng)
    eng.forward()
    with pytest.raises(api.DemError):
        E.backward()
    v2 = ds.verts.clone().requires_grad_(True)
    E2 = api.contact_energy(v2, eng)
    E2.backward()
    assert float(v2.grad.abs().max()) > 0


def _sub_contacts(cb, ti, tj):
    """A contact list made of the given (ti, tj) device tensors (the adjoint
    reads the triangle pair and the count only; other buffers are the
    originals, unread)."""
    n = int(ti.numel())
    return api.ContactBuffers(max(1, n), cb.pi, cb.pj, ti.contiguous(), tj.contiguous(), cb.d, cb.x, cb.n,
                              torch.tensor([n], dtype=torch.int32, device=ti.device))


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_backward_depends_on_the_contact_set_only(prec):
    """dE/dv is a sum over contacts: a shuffled contact list gives the same
    gradient and energy up to rounding, and a list split into a short head
    (1, 2, 3 or 5 contacts: a thread's group of consecutive contacts cut
    short) and the rest gives two parts that add up to the whole."""
    if prec == "f32":
        scene = sg.two_spheres(4, [2, 3, 4], "f32", sep=2.03, stream_id=44, name="g32")
        rtol = 1e-5
    else:
        scene = sg.two_spheres(3, [1, 2, 3], "f64", sep=2.03, stream_id=43, name="g64")
        rtol = 1e-12
    ds = api.DeviceScene(scene, device="cuda:0")
    eng = api.ContactEngine(ds, api.make_params("hier"), energy_k=1e4)
    assert eng.run() == 0
    n = eng.count()
    assert n > 100
    full = eng.contacts

    def grad_of(cb):
        g = torch.zeros(3, ds.n_verts, dtype=ds.dtype, device="cuda:0")
        eng.contacts = cb
        try:
            eng.backward(g, energy=True)
            torch.cuda.synchronize()
        finally:
            eng.contacts = full
        assert eng.check() == 0
        return g.double().cpu().numpy(), float(eng.energy_bwd.item())

    g0, e0 = grad_of(full)
    gmax = np.abs(g0).max()
    assert gmax > 0 and e0 > 0
    ti, tj = full.ti[:n], full.tj[:n]
    perm = torch.as_tensor(np.random.default_rng(7).permutation(n), device="cuda:0")
    g1, e1 = grad_of(_sub_contacts(full, ti[perm], tj[perm]))
    assert np.abs(g1 - g0).max() <= rtol * gmax
    assert abs(e1 - e0) <= rtol * e0
    for m in (1, 2, 3, 5):
        gh, eh = grad_of(_sub_contacts(full, ti[:m], tj[:m]))
        gr, er = grad_of(_sub_contacts(full, ti[m:], tj[m:]))
        assert np.abs(gh).max() > 0
        assert np.abs(gh + gr - g0).max() <= rtol * gmax, m
        assert abs(eh + er - e0) <= rtol * e0, m


# ------------------------------------------------------------------ failure handling
def test_contact_overflow_reports_needed_count():
    scene = sg.two_spheres(3, [1, 2, 3], "f32", sep=2.03, stream_id=45, name="ovf")
    ds = api.DeviceScene(scene, device="cuda:0")
    eng = api.ContactEngine(ds, api.make_params("hier"), contact_capacity=7)
    eng.forward()
    status = eng.check()
    assert status & _abi.DEM_DEV_CONTACT_OVERFLOW
    need = eng.count()
    eng2 = api.ContactEngine(ds, api.make_params("hier"))
    assert eng2.run() == 0 and eng2.count() == need > 7


def test_zero_iterations_same_contacts():
    """N_it = 0 leaves only the centroid/vertex bound: more fallback work,
    same contact set."""
    scene = sg.two_spheres(3, [1, 2, 3], "f32", sep=2.03, stream_id=46, name="nit0")
    ds, e4, r4 = run(scene, "hier")
    _, e0, r0 = run(scene, "hier", n_iter=0)
    assert set(keyed(ds, r4)) == set(keyed(ds, r0))
    assert e0.stats_dict()["near"] >= e4.stats_dict()["near"]


# ------------------------------------------------------------------ graphs
def test_graph_replay_matches_eager():
    scene = sg.two_spheres(4, [1, 2, 3, 4], "f32", sep=2.03, stream_id=47, name="graph")
    ds = api.DeviceScene(scene, device="cuda:0")
    eng = api.ContactEngine(ds, api.make_params("hier"), energy_k=1e4)
    eng.run()
    grad = torch.zeros(3, ds.n_verts, dtype=ds.dtype, device="cuda:0")
    eng.backward(grad)
    torch.cuda.synchronize()
    n_ref, e_ref, g_ref = eng.count(), float(eng.energy.item()), grad.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        grad.zero_()
        eng.forward()
        eng.backward(grad)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        grad.zero_()
        eng.forward()
        eng.backward(grad)
    for _ in range(3):
        junk = torch.randn(1000, device="cuda:0").sum()  # eager work between replays
        g.replay()
        torch.cuda.synchronize()
        assert eng.check() == 0
        assert eng.count() == n_ref
        assert abs(float(eng.energy.item()) - e_ref) <= 1e-9 * e_ref
        assert torch.allclose(grad, g_ref, rtol=1e-5, atol=1e-6 * float(g_ref.abs().max()))
        del junk


# ------------------------------------------------------------------ poses
def _rot90z():
    return np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])


def test_pose_exact_rotation_matches_oracle():
    """A 90-degree rotation applied in the flatten kernel is exact in FP32:
    contacts must match the oracle on the rotated coordinates."""
    scene = sg.two_spheres(4, [1, 2, 3, 4], "f32", sep=2.03, stream_id=48, name="pose90")
    ds = api.DeviceScene(scene, device="cuda:0")
    R = _rot90z()
    pose = np.concatenate([np.tile(R.reshape(1, 9), (ds.n_particles, 1)), np.zeros((ds.n_particles, 3))], 1)
    ds.set_pose(torch.as_tensor(pose, dtype=ds.dtype, device="cuda:0").contiguous())
    eng = api.ContactEngine(ds, api.make_params("hier"))
    assert eng.run() == 0
    res = eng.result()
    rotated = [scene.world(p) @ R.T for p in range(len(scene.particles))]
    fs = oracle.fine_scene(scene, verts_override=rotated)
    ref = oracle.find_contacts(fs)
    n, _, _ = compare_sets(scene, ds, res, ref, TOL["f32"], fs=fs)
    assert n > 500


def test_pose_small_rigid_motion_within_rounding():
    """Random small rigid motions (as in the fwd+bwd benchmark) applied in
    the flatten kernel, against the oracle on the exact FP64 rigid images;
    the bar adds the FP32 rounding of the transform (8 ulp of the largest
    coordinate) to the distance tolerance and the threshold band."""
    scene = sg.lattice_scene(3, stream_id=49, s_choices=(2, 3))
    ds = api.DeviceScene(scene, device="cuda:0")
    P = ds.n_particles
    Rs, ts = sg.rigid_perturbations(P, 4, stream_id=49)
    k = 3
    centres = np.array([p.centre for p in scene.particles])
    shift = centres + ts[k] - np.einsum("pij,pj->pi", Rs[k], centres)
    pose = np.concatenate([Rs[k].reshape(P, 9), shift], 1)
    ds.set_pose(torch.as_tensor(pose, dtype=ds.dtype, device="cuda:0").contiguous())
    eng = api.ContactEngine(ds, api.make_params("hier"))
    assert eng.run() == 0
    res = eng.result()
    moved = [(scene.world(p) - centres[p]) @ Rs[k][p].T + centres[p] + ts[k][p] for p in range(P)]
    fs = oracle.fine_scene(scene, verts_override=moved)
    ref = oracle.find_contacts(fs)
    cmax = max(np.abs(m).max() for m in moved)
    extra = 8 * 2.0 ** -24 * cmax
    tol = dict(TOL["f32"])
    tol["a"] = TOL["f32"]["a"]
    tol["band"] = TOL["f32"]["band"] + 2 * extra
    # distances: add the transform rounding as an absolute term
    g = keyed(ds, res)
    o = oracle_keyed(scene, ref)
    common = sorted(set(g) & set(o))
    dg = np.array([res["d"][g[c]] for c in common])
    dr = np.array([ref["d"][o[c]] for c in common])
    h = np.array([longest_edge(*pair_geom(fs, *c)) for c in common])
    assert np.all(np.abs(dg - dr) <= 1e-5 * dr + 1e-6 * h + 2 * extra)
    for key in set(o) - set(g):
        assert abs(ref["d"][o[key]] - 0.1) <= tol["band"]
    for key in set(g) - set(o):
        assert abs(oracle.tri_tri(*pair_geom(fs, *key))["d"] - 0.1) <= tol["band"]
    assert len(common) > 100


def test_certified_hybrid_matches_exact_fallback():
    """certify=1 (iterate + snap + certificate, fallback for the rest) and
    certify=0 (exact distance for every near pair) give the same contacts,
    and both meet the oracle bar."""
    scene = sg.two_spheres(4, [1, 2, 3, 4], "f32", sep=2.03, stream_id=50, name="cert")
    ds, e1, r1 = run(scene, "hier", certify=1)
    _, e0, r0 = run(scene, "hier", certify=0)
    st = e1.stats_dict()
    assert st["certified"] > 0 and st["certified"] + st["fallback"] == st["near"]
    assert e0.stats_dict()["certified"] == 0
    ref = oracle.find_contacts(oracle.fine_scene(scene))
    compare_sets(scene, ds, r1, ref, TOL["f32"])
    compare_sets(scene, ds, r0, ref, TOL["f32"])


@pytest.mark.parametrize("half_depths", [2, 32])
def test_reduced_precision_iteration_keeps_the_contacts(half_depths):
    """Newton iterations in half precision on the coarse depths (or all of
    them): the bound stays FP32, so the contact set and its exact distances
    are those of the FP32 iteration; pruning changes little."""
    scene = sg.two_spheres_s5_hier()
    ds = api.DeviceScene(scene, device="cuda:0")
    e32 = api.ContactEngine(ds, api.make_params("hier"))
    assert e32.run() == 0
    r32, s32 = e32.result(), e32.stats_dict()
    e16 = api.ContactEngine(ds, api.make_params("hier", half_depths=half_depths))
    assert e16.run() == 0
    r16, s16 = e16.result(), e16.stats_dict()
    k32 = sorted(zip(r32["ti"].tolist(), r32["tj"].tolist(), r32["d"].tolist()))
    k16 = sorted(zip(r16["ti"].tolist(), r16["tj"].tolist(), r16["d"].tolist()))
    assert len(k32) > 100 and k32 == k16
    # and against the oracle directly
    n, _, _ = compare_sets(scene, ds, r16, oracle.find_contacts(oracle.fine_scene(scene)), TOL["f32"])
    assert n > 100
    say(f"evals fp32 {s32['evals'][:3].tolist()} half {s16['evals'][:3].tolist()}")
    assert s16["evals"].sum() <= 1.05 * s32["evals"].sum()


# ------------------------------------------------------------------ deterministic order
def _keys(r):
    return (r["ti"].astype(np.int64) << 32) | r["tj"].astype(np.int64)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_deterministic_contact_order(prec):
    """dem_sort_contacts: the contacts come in strictly increasing (ti, tj)
    order, the arrays are identical on every run, and set and values are the
    unsorted forward's."""
    if prec == "f32":
        scene = sg.two_spheres(4, [2, 3, 4], "f32", 2.02, 4, "two_spheres_s4_f32")
    else:
        scene = sg.two_spheres_s3_f64()
    ds = api.DeviceScene(scene, device="cuda:0")
    plain = api.ContactEngine(ds, api.make_params("hier"))
    assert plain.run() == 0
    r0 = plain.result()
    det = api.ContactEngine(ds, api.make_params("hier"), deterministic=True)
    runs = []
    for _ in range(3):
        assert det.run() == 0
        runs.append(det.result())
    k = _keys(runs[0])
    assert len(k) > 100 and np.all(np.diff(k) > 0)
    for r in runs[1:]:
        for f in ("pi", "pj", "ti", "tj", "d", "x", "n"):
            assert np.array_equal(r[f], runs[0][f]), f
    o = np.argsort(_keys(r0))
    assert np.array_equal(_keys(r0)[o], k)
    for f in ("pi", "pj", "d", "x", "n"):
        assert np.array_equal(r0[f][o], runs[0][f]), f


def test_deterministic_order_in_a_graph():
    """Forward + sort captured in one HIP graph, replayed twice with eager work
    in between: the same arrays as the eager deterministic forward."""
    scene = sg.two_spheres(4, [2, 3, 4], "f32", 2.02, 4, "two_spheres_s4_f32")
    ds = api.DeviceScene(scene, device="cuda:0")
    eng = api.ContactEngine(ds, api.make_params("hier"), deterministic=True)
    assert eng.run() == 0
    ref = eng.result()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            eng.forward()
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(2):
        eng.forward()  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert eng.check() == 0
        got = eng.result()
        for f in ("pi", "pj", "ti", "tj", "d", "x", "n"):
            assert np.array_equal(got[f], ref[f]), (rep, f)


def test_understated_depth_flags_bad_tree():
    """A scene whose n_levels_max is one below its trees' depth: surrogate
    pairs survive the last depth launched and their pairs below are never
    tested, which the call must report (DEM_DEV_BAD_TREE) rather than return
    a short contact set.  Checked for the deepest depth's own kernel variant
    (256-thread blocks) and the general kernel (128-thread blocks)."""
    scene = sg.two_spheres(3, [1, 2, 3], "f32", sep=2.03, stream_id=47, name="depth")
    for block in (256, 128):
        ds = api.DeviceScene(scene, device="cuda:0")
        ok = api.ContactEngine(ds, api.make_params("hier", block=block))
        ok.forward()
        assert ok.check() == 0
        assert ds.n_levels_max >= 2
        ds.n_levels_max -= 1
        ds._refresh()
        eng = api.ContactEngine(ds, api.make_params("hier", block=block))
        eng.forward()
        say(f"[gpu-test] understated depth, block {block}: status {eng.check():#x}")
        assert eng.check() & _abi.DEM_DEV_BAD_TREE


def test_deepest_depth_variant_matches_general_kernel():
    """The deepest depth runs its own kernel variant (near pairs only, checks
    every eighth round) with 256-thread blocks and the general kernel with
    128-thread blocks: the same contacts with bit-identical distances and the
    same evaluation and survivor counts at every depth."""
    scene = sg.two_spheres(4, [1, 2, 3, 4], "f32", sep=2.03, stream_id=48, name="leaf")
    out = {}
    for block in (256, 128):
        ds = api.DeviceScene(scene, device="cuda:0")
        eng = api.ContactEngine(ds, api.make_params("hier", block=block))
        assert eng.run() == 0
        r = eng.result()
        st = eng.stats_dict()
        L = ds.n_levels_max
        out[block] = ({(int(a), int(b)): float(d) for a, b, d in zip(r["ti"], r["tj"], r["d"])},
                      np.asarray(st["evals"])[:L].tolist(), np.asarray(st["survivors"])[:L].tolist())
        say(f"[gpu-test] deepest-depth variant, block {block}: {len(out[block][0])} contacts, "
            f"evals {out[block][1]}")
    assert len(out[256][0]) > 100
    assert out[256][0] == out[128][0]
    assert out[256][1] == out[128][1] and out[256][2] == out[128][2]
