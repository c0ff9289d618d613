"""The persistent descent (one launch for seeding, every depth and the lazy
fine flattening, with a device work queue and grid barriers) against the
per-depth launches and the FP64 oracle.  Both run the same arithmetic on
every triangle pair, so the contact sets, distances and per-depth
evaluation counts must be identical; only the order of the work (and so of
the contacts) differs."""
import numpy as np
import pytest
import torch

import oracle
import scenegen as sg
from paper_2105_12415_amd import _abi, api

from test_gpu_parity import TOL, compare_sets, say

pytestmark = pytest.mark.gpu


def _run(ds, persistent, **kw):
    eng = api.ContactEngine(ds, api.make_params("hier", persistent=persistent, **kw), energy_k=1e4,
                            contact_capacity=1 << 21)
    assert eng.run() == 0
    assert eng.p.persistent == persistent  # no fall-back happened
    return eng, eng.result()


def _sorted(res):
    o = np.lexsort((res["tj"], res["ti"]))
    return {k: np.asarray(res[k])[o] for k in ("pi", "pj", "ti", "tj", "d", "x", "n")}


def _same(ra, rb):
    a, b = _sorted(ra), _sorted(rb)
    for k in a:
        assert np.array_equal(a[k], b[k]), k
    return len(a["d"])


def _scene(name):
    if name == "s4_levels_f32":
        return sg.two_spheres(4, [0, 1, 2, 3, 4], "f32", sep=2.03, stream_id=61, name=name)
    if name == "s3_levels_f64":
        return sg.two_spheres(3, [1, 2, 3], "f64", sep=2.03, stream_id=62, name=name)
    if name == "lattice27_depths_2_4":
        return sg.lattice_scene(3, stream_id=63, s_choices=(2, 3, 4))
    if name == "tori_kmeans_f32":
        from generic_mesh import two_tori_scene
        return two_tori_scene("f32")[0]
    raise KeyError(name)


@pytest.mark.parametrize("name", ["s4_levels_f32", "s3_levels_f64", "lattice27_depths_2_4", "tori_kmeans_f32"])
def test_persistent_matches_per_depth_launches(name):
    scene = _scene(name)
    ds = api.DeviceScene(scene, device="cuda:0")
    e0, r0 = _run(ds, 0)
    e1, r1 = _run(ds, 1)
    n = _same(r0, r1)
    s0, s1 = e0.stats_dict(), e1.stats_dict()
    assert np.array_equal(s0["evals"], s1["evals"]) and s0["near"] == s1["near"]
    # records the lazy flattening wrote: the same parents survive either way
    assert s0["fine_records"] == s1["fine_records"] <= ds.n_tris
    assert abs(r0["energy"] - r1["energy"]) <= 1e-12 * abs(r0["energy"]) + 1e-300
    say(f"[gpu-test] {name}: {n} contacts, evals {s1['evals'][:ds.n_levels_max].tolist()}")
    assert n > 50


def test_persistent_against_oracle_two_spheres_s5():
    scene = sg.two_spheres_s5_hier()
    ds = api.DeviceScene(scene, device="cuda:0")
    _, res = _run(ds, 1)
    n, _, _ = compare_sets(scene, ds, res, oracle.find_contacts(oracle.fine_scene(scene)), TOL["f32"])
    assert n > 1000


def test_persistent_dense_mode_and_half_depths():
    """Every fine pair through the persistent descent (dense distances), and
    the reduced-precision iteration on its coarse depths."""
    scene = sg.two_spheres(2, [0, 1, 2], "f32", sep=2.03, stream_id=64, name="dense_p")
    ds = api.DeviceScene(scene, device="cuda:0")
    _, r0 = _run(ds, 0, dense_distance=1)
    _, r1 = _run(ds, 1, dense_distance=1)
    assert _same(r0, r1) == 320 * 320
    scene = sg.two_spheres_s5_hier()
    ds = api.DeviceScene(scene, device="cuda:0")
    _, h0 = _run(ds, 0, half_depths=2)
    _, h1 = _run(ds, 1, half_depths=2)
    _same(h0, h1)


def test_persistent_full_lattice():
    """The 1000-sphere lattice: persistent and per-depth descents give the
    same contacts (6.5 M) and evaluation counts."""
    scene = sg.lattice1000()
    ds = api.DeviceScene(scene, device="cuda:0")
    e0, r0 = _run(ds, 0)
    e1, r1 = _run(ds, 1)
    n = _same(r0, r1)
    assert n > 10 ** 6
    assert np.array_equal(e0.stats_dict()["evals"], e1.stats_dict()["evals"])


def test_persistent_in_a_graph():
    """Forward + backward with the persistent descent captured in one HIP
    graph and replayed, with eager work in between: every replay equals the
    eager step."""
    scene = sg.two_spheres(4, [1, 2, 3, 4], "f32", sep=2.03, stream_id=65, name="graph_p")
    ds = api.DeviceScene(scene, device="cuda:0")
    eng = api.ContactEngine(ds, api.make_params("hier", persistent=1), energy_k=1e4)
    assert eng.run() == 0 and eng.p.persistent == 1
    grad = torch.zeros(3, ds.n_verts, dtype=ds.dtype, device="cuda:0")
    eng.backward(grad)
    torch.cuda.synchronize()
    n_ref, e_ref, g_ref = eng.count(), float(eng.energy.item()), grad.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            grad.zero_()
            eng.forward()
            eng.backward(grad)
    torch.cuda.current_stream().wait_stream(s)
    for _ in range(3):
        junk = torch.randn(1000, device="cuda:0").sum()
        g.replay()
        torch.cuda.synchronize()
        assert eng.check() == 0
        assert eng.count() == n_ref
        assert abs(float(eng.energy.item()) - e_ref) <= 1e-9 * e_ref
        assert torch.allclose(grad, g_ref, rtol=1e-5, atol=1e-6 * float(g_ref.abs().max()))
        del junk


def test_persistent_barrier_give_up_falls_back():
    """A grid barrier that gives up after one poll (a limit set from the
    host) reports DEM_DEV_STALLED instead of waiting; run() then repeats the
    call with one launch per depth and gets the full contact set."""
    scene = sg.two_spheres(4, [0, 1, 2, 3, 4], "f32", sep=2.03, stream_id=66, name="stall")
    ds = api.DeviceScene(scene, device="cuda:0")
    _, ref = _run(ds, 0)
    eng = api.ContactEngine(ds, api.make_params("hier", persistent=1, persistent_spins=1), energy_k=1e4,
                            contact_capacity=1 << 21)
    eng.forward()
    status = eng.check()
    say(f"[gpu-test] one-poll barriers: status {status:#x}")
    assert eng.run() == 0
    if status & _abi.DEM_DEV_STALLED:
        assert eng.p.persistent == 0
    _same(ref, eng.result())
