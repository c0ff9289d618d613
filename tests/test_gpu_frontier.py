"""GPU parity of the persistent active sets (dem_frontier_init and
dem_frontier_step through the C ABI) against the oracle's Frontier
(Section 5.3, Algorithm 6, pairwise reading, with the memory set).

- With p.prune_exact = 1 both sides decide "in range" with the exact distance,
  so the active sets must agree leaf for leaf (triangle ids, memory flags and
  depth, in the same depth-first order) after every step, and each step's
  contacts and widening / narrowing counts must agree.  The FP64 runs build
  the surrogate epsilons without slack, so both sides compare against the
  same thresholds up to rounding; every oracle step asserts that no decision
  lies within 1e-9 (relative) of its threshold, which makes the comparison
  well posed.
- With the iteration's lower bound (the default) the active sets may hold
  more pairs than the exact ones; the tests check what holds for any correct
  run: the leaves cover every fine pair exactly once, at most one level is
  unfolded per step, each step's contacts are true contacts, and a fixed
  point reports the all-pairs contact set (Lemma 1).
Distance and set tolerances are those of test_gpu_parity.
"""
import numpy as np
import pytest
import torch

import frontier_scenes as fsc
import oracle
import scenegen as sg
from oracle.frontier import Frontier
from paper_2105_12415_amd import _abi, api
from test_gpu_parity import TOL, compare_sets, keyed, longest_edge, oracle_keyed, pair_geom, say

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _announce(request):
    say(f"[gpu-test] {request.node.nodeid}")
    yield


def rows(eng):
    """(n, 4): t_i, t_j, flags, pair depth of the GPU's current leaves."""
    L = eng.leaves()
    return np.stack([L[:, 0], L[:, 1], L[:, 2], (L[:, 3] >> 17) & 31], 1)


def set_world(ds, scene):
    W = np.concatenate([scene.world(p) for p in range(len(scene.particles))])
    ds.verts.copy_(torch.as_tensor(W.T.copy(), dtype=ds.dtype))


def gpu_contacts(eng):
    r = eng.result()
    return sorted(zip(r["ti"].tolist(), r["tj"].tolist())), r


def step_both(eng, of, sc, ds):
    set_world(ds, sc)
    ro = of.step(oracle.tree(sc))
    status = eng.run_step()
    assert status == 0, hex(status)
    return ro


# ------------------------------------------------------------------ hand-built trees
@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("build", ["two_level", "three_level"])
def test_hand_sequences_match_oracle(prec, build):
    sc = getattr(fsc, build)(prec, fsc.NEAR)
    ds = api.DeviceScene(sc, device="cuda:0")
    t = oracle.tree(sc)
    assert np.array_equal(ds.tri_verts_host, t.tris)  # one numbering on both sides
    eng = api.FrontierEngine(ds, api.make_params("hier", prune_exact=1))
    eng.init()
    of = Frontier(t)
    assert np.array_equal(rows(eng), of.leaves())
    for where in (fsc.NEAR, fsc.NEAR, fsc.NEAR, fsc.FAR, fsc.FAR, fsc.NEAR, fsc.NEAR, fsc.FAR, fsc.NEAR):
        fsc.move_b(sc, where)
        ro = step_both(eng, of, sc, ds)
        assert np.array_equal(rows(eng), of.leaves()), (where, rows(eng), of.leaves())
        got, r = gpu_contacts(eng)
        assert got == sorted(zip(ro["a"].tolist(), ro["b"].tolist()))
        s = eng.stats_dict()
        assert (s["frontier_unfolded"], s["frontier_collapsed"]) == (ro["unfolded"], ro["collapsed"])
        assert s["frontier_leaves"] == ro["leaves_in"]


# ------------------------------------------------------------------ spheres, exact decisions
def _spheres(prec, sep=2.02):
    return sg.two_spheres(3, [1, 2, 3], prec, sep, 11, "two_spheres_s3_levels123")


def _place(sc, rot0, sep, angle=0.0):
    """Particle 1 at (sep, 0, 0), turned by `angle` about z from its start."""
    c, s = np.cos(angle), np.sin(angle)
    sc.particles[1].centre = np.array([sep, 0.0, 0.0])
    sc.particles[1].rot = np.array([[c, -s, 0], [s, c, 0], [0, 0, 1.0]]) @ rot0


def test_spheres_exact_frontier_matches_oracle_fp64():
    sc = _spheres("f64")
    rot0 = sc.particles[1].rot.copy()
    ds = api.DeviceScene(sc, device="cuda:0", coord_scale=1e-300, rel_slack=0.0)
    eng = api.FrontierEngine(ds, api.make_params("hier", prune_exact=1))
    eng.init()
    of = Frontier(oracle.tree(sc))
    # contact, apart, back, apart, then a slow roll of particle 1 about z
    script = [(2.02, 0.0)] * 5 + [(6.0, 0.0)] * 4 + [(2.02, 0.0)] * 5 + [(6.0, 0.0)] * 3
    script += [(2.0, 0.01 * k) for k in range(1, 7)]
    tol = TOL["f64"]
    n_changes = 0
    for k, (sep, ang) in enumerate(script):
        _place(sc, rot0, sep, ang)
        ro = step_both(eng, of, sc, ds)
        assert ro["margin"] > 1e-9, ("a decision lies on its threshold", k, ro["margin"])
        assert np.array_equal(rows(eng), of.leaves()), k
        s = eng.stats_dict()
        assert (s["frontier_unfolded"], s["frontier_collapsed"]) == (ro["unfolded"], ro["collapsed"]), k
        n_changes += ro["unfolded"] + ro["collapsed"]
        got, r = gpu_contacts(eng)
        assert got == sorted(zip(ro["a"].tolist(), ro["b"].tolist())), k
        if len(ro["a"]):
            dg = r["d"][np.lexsort((r["tj"], r["ti"]))]
            dr = ro["d"][np.lexsort((ro["b"], ro["a"]))]
            assert np.all(np.abs(dg - dr) <= tol["r"] * dr + tol["a"] * 0.25), k
    assert n_changes > 10


# ------------------------------------------------------------------ spheres, iteration decisions
def fine_sets(ds):
    cb = ds.child_begin.cpu().numpy()
    cc = ds.child_count.cpu().numpy()
    memo = {}

    def desc(x):
        if x in memo:
            return memo[x]
        if cc[x] == 0:
            out = np.array([x], np.int64)
        else:
            out = np.concatenate([desc(int(k)) for k in range(cb[x], cb[x] + cc[x])])
        memo[x] = out
        return out
    return desc


def assert_cover(ds, L, desc):
    """The leaves of every candidate pair cover its fine pairs exactly once."""
    got = np.sort(np.concatenate([(desc(int(a))[:, None] * (1 << 32) + desc(int(b))[None, :]).ravel()
                                  for a, b in L[:, :2]]))
    want = []
    for pi, pj in ds.pairs_host:
        Fi = np.arange(ds.fine_begin_host[pi], ds.fine_begin_host[pi] + ds.fine_count_host[pi])
        Fj = np.arange(ds.fine_begin_host[pj], ds.fine_begin_host[pj] + ds.fine_count_host[pj])
        want.append((Fi[:, None] * (1 << 32) + Fj[None, :]).ravel())
    assert np.array_equal(got, np.sort(np.concatenate(want)))


def check_true_contacts(sc, ds, res, ref, tol, fs):
    """Every GPU contact is an oracle contact (or within the band of delta),
    at the oracle's distance."""
    g = keyed(ds, res)
    o = oracle_keyed(sc, ref)
    delta = 2 * sc.particles[0].eps0
    for key in set(g) - set(o):
        d = oracle.tri_tri(*pair_geom(fs, *key))["d"]
        assert abs(d - delta) <= tol["band"], ("spurious contact", key, d)
    common = sorted(set(g) & set(o))
    dg = np.array([res["d"][g[k]] for k in common])
    dr = np.array([ref["d"][o[k]] for k in common])
    h = np.array([longest_edge(*pair_geom(fs, *k)) for k in common])
    assert np.all(np.abs(dg - dr) <= tol["r"] * dr + tol["a"] * h)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_spheres_iterate_frontier_properties(prec):
    sc = _spheres(prec)
    ds = api.DeviceScene(sc, device="cuda:0")
    eng = api.FrontierEngine(ds)
    eng.init()
    desc = fine_sets(ds)
    fs = oracle.fine_scene(sc)
    ref = oracle.find_contacts(fs)
    tol = TOL[prec]
    for k in range(1, 16):
        assert eng.run_step() == 0
        L = rows(eng)
        assert_cover(ds, L, desc)
        assert L[:, 3].max() <= k
        res = eng.result()
        check_true_contacts(sc, ds, res, ref, tol, fs)
        s = eng.stats_dict()
        if s["frontier_unfolded"] == 0 and s["frontier_collapsed"] == 0:
            break
    else:
        pytest.fail("no fixed point")
    n_common, _, _ = compare_sets(sc, ds, res, ref, tol, fs)
    assert n_common > 20
    say(f"fixed point after {k} steps: {len(L)} leaves, {n_common} contacts")


def test_frontier_backward_matches_descent_at_fixed_point():
    sc = _spheres("f32")
    ds = api.DeviceScene(sc, device="cuda:0")
    eng = api.FrontierEngine(ds)
    eng.init()
    for _ in range(16):
        eng.run_step()
        s = eng.stats_dict()
        if s["frontier_unfolded"] == 0 and s["frontier_collapsed"] == 0:
            break
    g1 = torch.zeros(3, ds.n_verts, dtype=ds.dtype, device=ds.device)
    eng.backward(g1, energy=True)
    ce = api.ContactEngine(ds)
    ce.run()
    g2 = torch.zeros_like(g1)
    ce.backward(g2, energy=True)
    torch.cuda.synchronize()
    assert eng.count() == ce.count() > 20
    scale = float(g2.abs().max())
    assert float((g1 - g2).abs().max()) <= 1e-4 * scale
    assert abs(float(eng.energy_bwd.item()) - float(ce.energy_bwd.item())) <= 1e-5 * float(ce.energy_bwd.item())


# ------------------------------------------------------------------ edge cases
def test_frontier_without_candidate_pairs():
    sc = _spheres("f32")
    sc.pairs = np.zeros((0, 2), np.int32)
    ds = api.DeviceScene(sc, device="cuda:0")
    eng = api.FrontierEngine(ds)
    eng.init()
    assert eng.state_host()[1] == 0
    assert eng.run_step() == 0
    assert eng.count() == 0 and len(eng.leaves()) == 0


def test_frontier_capacity_growth_keeps_the_sets():
    """Root pairs above the capacity (init grows it) and a widening step
    above it (the step is rerun on larger buffers) give the same active sets
    as a run with room to spare."""
    sc = _spheres("f32")
    ds = api.DeviceScene(sc, device="cuda:0")
    big = api.FrontierEngine(ds, capacity=1 << 22)
    big.init()
    small = api.FrontierEngine(ds, capacity=1000)
    small.init()
    assert small.capacity > 1000
    small_cap = small.capacity
    for _ in range(4):
        assert big.run_step() == 0
        assert small.run_step() == 0
        assert np.array_equal(big.leaves(), small.leaves())
        assert big.count() == small.count()
    assert small.capacity > small_cap


def test_frontier_steps_in_a_graph_match_eager_steps():
    """Frontier steps with per-step poses captured in one HIP graph and
    replayed give the same active sets and contacts as the same steps run
    eagerly (everything the step decides stays on the device)."""
    sc = _spheres("f32")
    P = len(sc.particles)
    Rs, ts = sg.rigid_perturbations(P, 6, max_shift=2e-2, max_angle=2e-2)
    centres = np.array([p.centre for p in sc.particles])
    shift = centres[None] + ts - np.einsum("kpij,pj->kpi", Rs, centres)
    poses = np.concatenate([Rs.reshape(6, P, 9), shift], 2)

    def engine():
        ds = api.DeviceScene(sc, device="cuda:0")
        eng = api.FrontierEngine(ds, capacity=1 << 20)
        eng.init()
        eng.run_to_fixed_point()
        return ds, eng

    pose_t = [torch.as_tensor(poses[k], dtype=torch.float32, device="cuda:0").contiguous() for k in range(6)]
    ds_a, a = engine()
    for k in range(1, 6):
        ds_a.set_pose(pose_t[k])
        assert a.run_step() == 0
    ds_b, b = engine()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            for k in range(1, 6):
                ds_b.set_pose(pose_t[k])
                b.step()
    torch.cuda.current_stream().wait_stream(s)
    # two replays, each against the same five steps run eagerly (with the
    # program's own eager work and synchronisation in between)
    for rep in range(2):
        if rep:
            for k in range(1, 6):
                ds_a.set_pose(pose_t[k])
                assert a.run_step() == 0
        g.replay()
        torch.cuda.synchronize()
        assert b.check() == 0
        assert np.array_equal(a.leaves(), b.leaves()), rep
        ra, rb = a.result(), b.result()
        assert sorted(zip(ra["ti"].tolist(), ra["tj"].tolist())) == sorted(zip(rb["ti"].tolist(), rb["tj"].tolist()))
    say(f"{len(a.leaves())} leaves, {len(ra['ti'])} contacts")


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_frontier_certified_settling_matches_exact(prec):
    """certify = 1 settles the frontier's fine pairs from the iterate where the
    separation bound certifies the distance (the rest by the exact distance):
    same fixed-point leaves and contact set as exact settling."""
    sc = _spheres(prec)
    out = []
    for cert in (0, 1):
        ds = api.DeviceScene(sc, device="cuda:0")
        eng = api.FrontierEngine(ds, api.make_params("hier", certify=cert))
        eng.init()
        eng.run_to_fixed_point()
        r = eng.result()
        out.append((eng.leaves(), dict(zip(zip(r["ti"].tolist(), r["tj"].tolist()), r["d"].tolist())), eng.stats_dict()))
    (l0, c0, s0), (l1, c1, s1) = out
    assert np.array_equal(l0, l1)
    band = TOL[prec]["band"]
    for key in set(c0) ^ set(c1):
        d = c0.get(key, c1.get(key))
        assert abs(d - 0.1) <= band, key
    common = set(c0) & set(c1)
    assert len(common) > 20
    r_, a_ = TOL[prec]["r"], TOL[prec]["a"]
    assert all(abs(c0[k] - c1[k]) <= 4 * (r_ * c0[k] + a_ * 0.2) for k in common)
    assert s1["certified"] > 0
