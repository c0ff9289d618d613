"""dem_find_contacts_noalloc (workspace in the library's static device
scratch) against dem_find_contacts (caller workspace) through the C ABI:
the same contact set with bit-identical distances, points and normals, and
the same energy, on two calls in a row, the second with a smaller input
(fewer triangles and pairs), so that what the first call left in the
scratch cannot leak into the second.
"""
import ctypes as C
import sys

import numpy as np
import pytest
import torch

import scenegen as sg
from paper_2105_12415_amd import _abi, api

pytestmark = pytest.mark.gpu

# level lists and near list sized so that the workspace fits the scratch
CAPS = dict(queue_capacity=1 << 19, near_capacity=1 << 21)


def say(msg):
    print(msg, file=sys.stderr, flush=True)


def stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def sorted_contacts(cb: api.ContactBuffers):
    n = int(cb.count.item()) & 0xFFFFFFFF
    assert n <= cb.capacity
    ti, tj = cb.ti[:n].cpu().numpy(), cb.tj[:n].cpu().numpy()
    order = np.lexsort((tj, ti))
    return {"pi": cb.pi[:n].cpu().numpy()[order], "pj": cb.pj[:n].cpu().numpy()[order],
            "ti": ti[order], "tj": tj[order], "d": cb.d[:n].cpu().numpy()[order],
            "x": cb.x[:, :n].cpu().numpy()[:, order], "n": cb.n[:, :n].cpu().numpy()[:, order]}


def run_both(scene):
    ds = api.DeviceScene(scene, device="cuda:0")
    eng = api.ContactEngine(ds, api.make_params("hier", **CAPS))
    eng.run()
    ref = sorted_contacts(eng.contacts)
    e_ref = float(eng.energy.item())

    L = _abi.lib()
    p = api.make_params("hier", queue_capacity=eng.p.queue_capacity, near_capacity=eng.p.near_capacity)
    p.energy_k = eng.p.energy_k
    need = L.dem_workspace_bytes(C.byref(ds.c), ds.n_pairs, C.byref(p))
    assert 0 < need <= _abi.DEM_SCRATCH_BYTES, need
    out = api.ContactBuffers.alloc(eng.contacts.capacity, ds.dtype, ds.device)
    out.count.fill_(12345)
    stats = torch.zeros(_abi.STATS_WORDS, dtype=torch.int64, device=ds.device)
    status = torch.full((1,), -1, dtype=torch.int32, device=ds.device)
    energy = torch.full((1,), -1.0, dtype=torch.float64, device=ds.device)
    cs = out.c()
    say(f"[noalloc] {scene.name}: {ds.n_tris} triangles, {ds.n_pairs} pairs, workspace {need} B")
    st = L.dem_find_contacts_noalloc(C.byref(ds.c), C.c_void_p(ds.pairs.data_ptr()), ds.n_pairs, C.byref(p),
                                     C.byref(cs), C.c_void_p(stats.data_ptr()), C.c_void_p(status.data_ptr()),
                                     C.c_void_p(energy.data_ptr()), stream())
    _abi.check(st, "dem_find_contacts_noalloc")
    torch.cuda.synchronize()
    assert int(status.item()) == 0, hex(int(status.item()) & 0xFFFFFFFF)
    got = sorted_contacts(out)
    assert len(got["ti"]) == len(ref["ti"]) > 0
    for k in ("pi", "pj", "ti", "tj", "d", "x", "n"):
        assert np.array_equal(got[k], ref[k]), k
    # energy: same per-contact terms, summed by atomics in another order
    assert abs(float(energy.item()) - e_ref) <= 1e-12 * abs(e_ref) + 1e-300
    s_got, s_ref = api._stats_dict(stats), eng.stats_dict()
    assert s_got["contacts"] == s_ref["contacts"] and s_got["near"] == s_ref["near"]
    # the gradient of the no-allocation call's contacts through their adjoint
    # rows, with no workspace at all, against the workspace call's
    g_ref = torch.zeros(3, ds.n_verts, dtype=ds.dtype, device=ds.device)
    eng.backward(g_ref)
    g = torch.zeros_like(g_ref)
    st = L.dem_contact_backward(C.byref(ds.c), C.byref(cs), float(p.energy_k), None, C.c_void_p(g.data_ptr()),
                                None, None, 0, C.c_void_p(status.data_ptr()), stream())
    _abi.check(st, "dem_contact_backward")
    torch.cuda.synchronize()
    assert int(status.item()) == 0, hex(int(status.item()) & 0xFFFFFFFF)
    gm = float(g_ref.abs().max())
    assert gm > 0
    assert float((g - g_ref).abs().max()) <= (1e-5 if ds.dtype == torch.float32 else 1e-12) * gm
    return len(got["ti"])


def test_noalloc_matches_workspace_call_twice():
    big = sg.two_spheres(5, [0, 1, 2, 3, 4, 5], "f32", sep=2.02, stream_id=31, name="noalloc_s5")
    n1 = run_both(big)
    small = sg.two_spheres(3, [0, 1, 2, 3], "f64", sep=2.03, stream_id=32, name="noalloc_s3_f64")
    n2 = run_both(small)
    say(f"[noalloc] contacts {n1} then {n2}")


def test_noalloc_rejects_oversize_workspace():
    scene = sg.two_spheres(3, [0, 1, 2, 3], "f32", sep=2.03, stream_id=33, name="noalloc_oversize")
    ds = api.DeviceScene(scene, device="cuda:0")
    p = api.make_params("hier", queue_capacity=1 << 24, near_capacity=1 << 24)
    out = api.ContactBuffers.alloc(1 << 12, ds.dtype, ds.device)
    status = torch.zeros(1, dtype=torch.int32, device=ds.device)
    cs = out.c()
    st = _abi.lib().dem_find_contacts_noalloc(C.byref(ds.c), C.c_void_p(ds.pairs.data_ptr()), ds.n_pairs,
                                              C.byref(p), C.byref(cs), None, C.c_void_p(status.data_ptr()),
                                              None, stream())
    assert st == _abi.DEM_ERR_CAPACITY
