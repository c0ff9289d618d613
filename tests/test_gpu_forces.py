"""GPU parity of dem_contact_forces (through the C ABI) against the oracle's
contact forces (Section 2 force law; merging of contact points closer than
eps, read as single linkage within a particle pair).

Both sides start from their own contact lists (GPU: dem_find_contacts;
oracle: its exact all-pairs search); contacts are matched by (particle pair,
fine triangle pair).  Merging is a threshold decision on point distances, so
the partition is compared with a band: every group the oracle forms from
pairs clearly closer than the radius (distance < r - tol) lies inside one GPU
group, and every GPU group lies inside one oracle group formed with
distance < r + tol (with no pair inside the band the partitions are equal).
Groups with the same members on both sides are compared value by value:
point and normal within a few units of the precision, force within 2e-4 K_s
(FP32) / 1e-9 K_s (FP64).  Per-particle force and torque are compared when
the partitions agree exactly.
"""
import numpy as np
import pytest
import torch

import oracle
import scenegen as sg
from oracle import forces as of
from paper_2105_12415_amd import api
from test_gpu_parity import keyed, oracle_keyed, say

pytestmark = pytest.mark.gpu

TOLF = {"f64": dict(band=1e-9, x=1e-12, f=1e-9), "f32": dict(band=1e-4, x=2e-6, f=2e-4)}


@pytest.fixture(autouse=True)
def _announce(request):
    say(f"[gpu-test] {request.node.nodeid}")
    yield


def _mass_centre(scene):
    mass = np.array([p.radius ** 3 for p in scene.particles])
    centre = np.array([p.centre for p in scene.particles])
    return mass, centre


def _components(n, edges):
    parent = list(range(n))

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x
    for a, b in edges:
        ra, rb = find(a), find(b)
        if ra != rb:
            parent[max(ra, rb)] = min(ra, rb)
    return np.array([find(i) for i in range(n)])


def run_both(scene, merge_scale=1.0, ds=None, eng=None):
    ds = ds or api.DeviceScene(scene, device="cuda:0")
    if eng is None:
        eng = api.ContactEngine(ds)
        assert eng.run() == 0
    res = eng.result()
    mass, centre = _mass_centre(scene)
    fe = api.ForceEngine(ds, eng.contacts.capacity)
    fe.run(eng.contacts, torch.as_tensor(mass, dtype=ds.dtype, device=ds.device),
           torch.as_tensor(centre.T.copy(), dtype=ds.dtype, device=ds.device), merge_scale=merge_scale)
    assert fe.check() == 0
    g = fe.result(len(res["d"]))
    fs = oracle.fine_scene(scene)
    ref = oracle.find_contacts(fs)
    o = of.contact_forces(fs, ref, mass, centre, merge=merge_scale > 0)
    return ds, res, g, fs, ref, o


def compare(scene, ds, res, g, fs, ref, o, prec, merge_scale=1.0):
    tol = TOLF[prec]
    gk = keyed(ds, res)
    ok = oracle_keyed(scene, ref)
    assert set(gk) == set(ok), "contact sets differ (these scenes have no contact in the threshold band)"
    keys = sorted(ok)
    n = len(keys)
    # GPU partition over the common keys
    g_lab = np.array([g["group"][gk[k]] for k in keys])
    assert np.all(g_lab >= 0) and np.all(g_lab < len(g["f"]))
    o_lab = np.array([o["labels"][ok[k]] for k in keys])
    # oracle points for the band construction
    x, *_ = of.contact_points(fs, ref)
    xo = x[[ok[k] for k in keys]]
    pair = np.array([k[:2] for k in keys])
    r = merge_scale * 0.05  # merge_scale * (eps_i + eps_j) / 2 with eps = 0.05
    strict, loose = [], []
    if merge_scale > 0:
        for pk in {tuple(p) for p in pair}:
            idx = np.nonzero((pair[:, 0] == pk[0]) & (pair[:, 1] == pk[1]))[0]
            d = np.linalg.norm(xo[idx][:, None] - xo[idx][None], axis=2)
            ii, jj = np.nonzero(np.triu(d < r + tol["band"] * r, 1))
            for a, b in zip(ii, jj):
                loose.append((idx[a], idx[b]))
                if d[a, b] < r - tol["band"] * r:
                    strict.append((idx[a], idx[b]))
    cs, cl = _components(n, strict), _components(n, loose)
    for comp in np.unique(cs):
        assert len(np.unique(g_lab[cs == comp])) == 1, "a clearly merged group was split"
    for grp in np.unique(g_lab):
        assert len(np.unique(cl[g_lab == grp])) == 1, "a GPU group joins points that are clearly apart"
    exact = len(strict) == len(loose)
    # same-member groups: values
    o_groups = {}
    for k, lab in enumerate(o_lab):
        o_groups.setdefault(lab, []).append(k)
    o_row = {lab: i for i, lab in enumerate(np.unique(o["labels"]))}
    n_cmp = 0
    for lab, members in o_groups.items():
        gl = np.unique(g_lab[members])
        if len(gl) != 1 or np.sum(g_lab == gl[0]) != len(members):
            continue
        gi, oi = int(gl[0]), o_row[lab]
        assert g["members"][gi] == len(members)
        assert np.allclose(g["x"][gi], o["x"][oi], atol=tol["x"] * 20), (g["x"][gi], o["x"][oi])
        assert np.allclose(g["n"][gi], o["n"][oi], atol=tol["x"] * 20)
        assert np.allclose(g["f"][gi], o["f"][oi], atol=tol["f"] * of.K_S), (g["f"][gi], o["f"][oi])
        n_cmp += 1
    assert n_cmp > 0
    if exact:
        scale = np.abs(o["force"]).max()
        assert np.allclose(g["force"], o["force"], atol=tol["f"] * of.K_S * max(1, n_cmp))
        assert np.allclose(g["torque"], o["torque"], atol=tol["f"] * of.K_S * max(1, n_cmp) * 3)
        assert scale > 0
    return n_cmp, exact


@pytest.mark.parametrize("merge_scale", [1.0, 0.0])
def test_forces_two_spheres_fp64(merge_scale):
    scene = sg.two_spheres_s3_f64()
    out = run_both(scene, merge_scale)
    n_cmp, exact = compare(scene, *out, "f64", merge_scale)
    say(f"{n_cmp} groups compared, partitions exact: {exact}")
    assert exact


@pytest.mark.parametrize("merge_scale", [1.0, 0.0])
def test_forces_two_spheres_s4_fp32(merge_scale):
    scene = sg.two_spheres(4, [2, 3, 4], "f32", 2.02, 4, "two_spheres_s4_f32")
    out = run_both(scene, merge_scale)
    n_cmp, exact = compare(scene, *out, "f32", merge_scale)
    say(f"{n_cmp} groups compared, partitions exact: {exact}")


def test_vertex_to_vertex_duplicates_merge_on_gpu():
    rng = np.random.default_rng(0)
    a = sg.bumped_sphere(rng, 0, 1.0, bump=0.0, rotate=False)
    b = sg.bumped_sphere(rng, 0, 1.0, bump=0.0, rotate=False)
    v = a.body[0] / np.linalg.norm(a.body[0])
    b.centre = (2.0 + 0.05) * v
    scene = sg.Scene("vv", [a, b], np.array([[0, 1]], np.int32), "f64")
    ds, res, g, fs, ref, o = run_both(scene)
    assert len(res["d"]) == 25 and len(g["f"]) == 1 and g["members"][0] == 25
    assert np.allclose(g["f"][0], -500.0 * np.sqrt(0.5) * v, atol=1e-9)  # masses 1, 1
    assert np.allclose(g["force"][0], -g["force"][1], atol=1e-12)


def test_forces_without_contacts():
    scene = sg.two_spheres(3, None, "f32", 3.0, 1, "apart")
    ds, res, g, fs, ref, o = run_both(scene)
    assert len(res["d"]) == 0 and len(g["f"]) == 0
    assert np.all(g["force"] == 0) and np.all(g["torque"] == 0)


def test_force_pass_in_a_graph_matches_eager():
    """Contacts + force pass captured in one HIP graph, replayed twice with
    eager work in between, against the eager pass (sums in different atomic
    order: force and torque within 1e-5 of their largest entry)."""
    scene = sg.two_spheres(4, [2, 3, 4], "f32", 2.02, 4, "two_spheres_s4_f32")
    ds = api.DeviceScene(scene, device="cuda:0")
    eng = api.ContactEngine(ds)
    assert eng.run() == 0
    mass, centre = _mass_centre(scene)
    m = torch.as_tensor(mass, dtype=ds.dtype, device=ds.device)
    c = torch.as_tensor(centre.T.copy(), dtype=ds.dtype, device=ds.device)
    fe = api.ForceEngine(ds, eng.contacts.capacity)
    fe.run(eng.contacts, m, c, with_group=False)
    assert fe.check() == 0
    ref = fe.result(0)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            eng.forward()
            fe.run(eng.contacts, m, c, with_group=False)
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(2):
        eng.forward()  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert fe.check() == 0 and eng.check() == 0
        got = fe.result(0)
        assert len(got["f"]) == len(ref["f"]) and sorted(got["members"].tolist()) == sorted(ref["members"].tolist())
        fmax = np.abs(ref["force"]).max()
        assert np.allclose(got["force"], ref["force"], atol=1e-5 * fmax)
        assert np.allclose(got["torque"], ref["torque"], atol=1e-5 * np.abs(ref["torque"]).max())
