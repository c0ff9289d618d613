"""Host-side checks of the C ABI: library loads, exports every declared
symbol, validates arguments, and builds conservative hierarchies.  No device
computation is launched here."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

import oracle
import scenegen as sg
from paper_2105_12415_amd import _abi, api

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "dem.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dem_[a-z_0-9]+)\s*\(", src)))


def test_header_symbols_exported():
    names = declared_functions()
    assert set(names) == set(_abi.EXPORTS)
    L = _abi.lib()
    for n in names:
        assert hasattr(L, n), n
    assert L.dem_version().decode().startswith("dem ")


def test_struct_sizes_match_header_layout():
    # dem_stats: 3 arrays of 32 + 4 scalars + 3 frontier counters, 8 bytes each
    assert C.sizeof(_abi.Stats) == 8 * (3 * 32 + 4 + 4)
    p = _abi.default_params()
    assert p.n_iter == 4 and p.mode == _abi.DEM_MODE_HIER and p.omega == 1.0
    assert list(p.level_grid) == [0] * _abi.DEM_MAX_LEVELS and list(p.level_batch) == [0] * _abi.DEM_MAX_LEVELS


def test_ctypes_layout_matches_c_compiler(tmp_path):
    """Every field offset and struct size of the binding equals what a C
    compiler makes of include/dem.h."""
    structs = {"dem_build_opts": _abi.BuildOpts, "dem_hierarchy": _abi.Hierarchy, "dem_scene": _abi.Scene,
               "dem_params": _abi.Params, "dem_contacts": _abi.Contacts, "dem_stats": _abi.Stats,
               "dem_frontier": _abi.Frontier, "dem_merged": _abi.Merged}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "dem.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f in py._fields_:
            lines.append(f'  printf("{cname} {f[0]} %zu\\n", offsetof({cname}, {f[0]}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.check_call(["gcc", "-std=c99", "-I", inc, str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe)]).decode().split("\n")
    seen = 0
    for line in out:
        if not line:
            continue
        cname, field, val = line.split()
        py = structs[cname]
        want = C.sizeof(py) if field == "size" else getattr(py, field).offset
        assert int(val) == want, (cname, field, int(val), want)
        seen += 1
    assert seen == sum(len(py._fields_) + 1 for py in structs.values())


def test_status_strings():
    L = _abi.lib()
    for s in (0, -1, -2, -3, -4, -5):
        assert L.dem_status_string(s)
    assert L.dem_status_string(0).decode() == "ok"


def _fake_scene(precision=_abi.DEM_F32):
    s = _abi.Scene()
    s.precision = precision
    s.n_verts, s.n_tris, s.n_particles, s.n_levels_max = 10, 20, 2, 3
    for f in ("verts", "tri_verts", "child_begin", "child_count", "tri_particle", "tri_eps",
              "root_begin", "root_count", "fine_begin", "fine_count"):
        setattr(s, f, 4096)  # never dereferenced by host-side validation
    s.pose = None
    return s


def test_workspace_bytes_and_validation():
    L = _abi.lib()
    s = _fake_scene()
    p = _abi.default_params()
    n32 = L.dem_workspace_bytes(C.byref(s), 1, C.byref(p))
    s64 = _fake_scene(_abi.DEM_F64)
    n64 = L.dem_workspace_bytes(C.byref(s64), 1, C.byref(p))
    assert n32 > 0 and n64 > n32
    bad = _fake_scene()
    bad.n_levels_max = 0
    assert L.dem_workspace_bytes(C.byref(bad), 1, C.byref(p)) == 0
    p2 = _abi.default_params()
    p2.block = 100
    assert L.dem_workspace_bytes(C.byref(s), 1, C.byref(p2)) == 0
    # find_contacts rejects bad arguments before touching the device
    out = _abi.Contacts()
    st = L.dem_find_contacts(C.byref(s), None, 1, C.byref(p), C.byref(out), None, 0, None, None,
                             None, None)
    assert st == _abi.DEM_ERR_ARG
    out.count = 4096
    out.capacity = 0
    st = L.dem_find_contacts(C.byref(s), C.c_void_p(4096), 1, C.byref(p), C.byref(out),
                             C.c_void_p(4096), 16, None, C.c_void_p(4096), None, None)
    assert st == _abi.DEM_ERR_CAPACITY
    st = L.dem_contact_backward(C.byref(s), C.byref(out), -1.0, None, C.c_void_p(4096), None,
                                C.c_void_p(4096), 1 << 20, C.c_void_p(4096), None)
    assert st == _abi.DEM_ERR_ARG
    # without adjoint rows the backward needs the forward's workspace (soup)
    out.ti = out.tj = 4096
    out.adjoint = None
    st = L.dem_contact_backward(C.byref(s), C.byref(out), 1.0, None, C.c_void_p(4096), None,
                                None, 0, C.c_void_p(4096), None)
    assert st == _abi.DEM_ERR_ARG
    st = L.dem_contact_backward(C.byref(s), C.byref(out), 1.0, None, C.c_void_p(4096), None,
                                C.c_void_p(4096), 16, C.c_void_p(4096), None)
    assert st == _abi.DEM_ERR_CAPACITY


def test_find_contacts_noalloc_validation():
    """dem_find_contacts_noalloc rejects bad arguments and workspaces beyond
    its static scratch before any device call."""
    L = _abi.lib()
    s = _fake_scene()
    p = _abi.default_params()
    out = _abi.Contacts()
    assert L.dem_find_contacts_noalloc(C.byref(s), None, 1, C.byref(p), C.byref(out), None, None, None,
                                       None) == _abi.DEM_ERR_ARG
    out.count = 4096
    out.capacity = 0
    # default capacities need 2 x 64 MiB of queues alone
    assert L.dem_workspace_bytes(C.byref(s), 1, C.byref(p)) > _abi.DEM_SCRATCH_BYTES
    assert L.dem_find_contacts_noalloc(C.byref(s), C.c_void_p(4096), 1, C.byref(p), C.byref(out), None,
                                       C.c_void_p(4096), None, None) == _abi.DEM_ERR_CAPACITY
    p.block = 100
    assert L.dem_find_contacts_noalloc(C.byref(s), C.c_void_p(4096), 1, C.byref(p), C.byref(out), None,
                                       C.c_void_p(4096), None, None) == _abi.DEM_ERR_ARG


def test_sort_contacts_sizing_and_validation():
    """dem_sort_contacts: workspace grows with the triangle count and the
    capacity; bad arguments are rejected before any device work."""
    L = _abi.lib()
    s = _fake_scene()
    n0 = L.dem_sort_contacts_workspace_bytes(C.byref(s), 0)
    n1 = L.dem_sort_contacts_workspace_bytes(C.byref(s), 1 << 20)
    assert 0 < n0 < n1
    assert L.dem_sort_contacts_workspace_bytes(C.byref(s), -1) == 0
    big = _fake_scene()
    big.n_tris = s.n_tris * 64
    assert L.dem_sort_contacts_workspace_bytes(C.byref(big), 0) > n0
    out = _abi.Contacts()
    assert L.dem_sort_contacts(C.byref(s), None, C.c_void_p(4096), n1, C.c_void_p(4096), None) == _abi.DEM_ERR_ARG
    out.count = 4096
    out.capacity = 1 << 20  # buffers missing
    assert L.dem_sort_contacts(C.byref(s), C.byref(out), C.c_void_p(4096), n1, C.c_void_p(4096),
                               None) == _abi.DEM_ERR_ARG
    out.capacity = 0
    assert L.dem_sort_contacts(C.byref(s), C.byref(out), C.c_void_p(4096), 16, C.c_void_p(4096),
                               None) == _abi.DEM_ERR_CAPACITY
    assert L.dem_sort_contacts(C.byref(s), C.byref(out), C.c_void_p(4096), n0, None, None) == _abi.DEM_ERR_ARG


def _levels(p):
    sizes = [len(l) for l in p.levels]
    offs = np.cumsum([0] + sizes)
    tris = np.concatenate(p.levels)
    parent = np.full(len(tris), -1, np.int32)
    for l in range(1, len(p.levels)):
        parent[offs[l]:offs[l + 1]] = p.parents[l] + offs[l - 1]
    return tris, parent, sizes


def test_hierarchy_matches_oracle_eps():
    s = sg.two_spheres(4, [0, 1, 2, 3, 4], "f32", stream_id=31, name="h")
    t = oracle.tree(s)
    n0 = 0
    for k, p in enumerate(s.particles):
        tris, parent, sizes = _levels(p)
        h = api.build_hierarchy(s.world(k), tris, parent, sizes, p.eps0)
        n = len(tris)
        assert np.allclose(h["eps"], t.eps[n0:n0 + n], rtol=1e-13, atol=1e-15)
        # stored epsilons never fall below the exact ones
        assert np.all(h["eps_f32"].astype(np.float64) >= h["eps"])
        assert np.all(h["eps_f64"] >= h["eps"])
        # child ranges partition each level below the root
        cc = h["child_count"]
        assert np.all(cc[:h["fine_begin"]] == 4) and np.all(cc[h["fine_begin"]:] == 0)
        lb = h["level_begin"]
        for l in range(len(sizes) - 1):
            cb = h["child_begin"][lb[l]:lb[l + 1]]
            assert np.array_equal(cb, lb[l + 1] + 4 * np.arange(sizes[l]))
        n0 += n


def test_hierarchy_rejects_malformed():
    p = sg.two_spheres(2, [1, 2], "f64", stream_id=32).particles[0]
    tris, parent, sizes = _levels(p)
    w = p.world()
    bad = parent.copy()
    bad[sizes[0]] = sizes[0] + 3  # parent outside the previous level
    with pytest.raises(_abi.DemError):
        api.build_hierarchy(w, tris, bad, sizes, 0.05)
    bad = parent.copy()
    bad[sizes[0]:sizes[0] + 4] = 1  # children of face 0 re-assigned: face 0 childless, 1 split
    with pytest.raises(_abi.DemError):
        api.build_hierarchy(w, tris, bad, sizes, 0.05)
    with pytest.raises(_abi.DemError):
        api.build_hierarchy(w, tris + 10 ** 6, parent, sizes, 0.05)
