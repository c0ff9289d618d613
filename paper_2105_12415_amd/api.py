"""Python binding of libdem: scene packing, the three C-ABI calls, autograd.

Everything that touches contact geometry runs in libdem's HIP kernels; this
module only packs host arrays into the library's layout, allocates device
buffers with torch, and passes pointers and the current torch stream.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

from . import _abi
from ._abi import DemError, check, lib


# ------------------------------------------------------------------ hierarchy
def build_hierarchy(verts: np.ndarray, tris: np.ndarray, parent: np.ndarray, level_sizes,
                    eps0: float, coord_scale: float = 0.0, rel_slack: float = 1e-6) -> dict:
    """dem_build_hierarchy on one particle; returns numpy copies of the blob."""
    V = np.ascontiguousarray(verts, np.float64).reshape(-1, 3)
    T = np.ascontiguousarray(tris, np.int32).reshape(-1, 3)
    P = np.ascontiguousarray(parent, np.int32).reshape(-1)
    S = np.ascontiguousarray(level_sizes, np.int32).reshape(-1)
    opts = _abi.BuildOpts(float(coord_scale), float(rel_slack))
    h = _abi.Hierarchy()
    st = lib().dem_build_hierarchy(V.ctypes.data_as(C.POINTER(C.c_double)), len(V),
                                   T.ctypes.data_as(C.POINTER(C.c_int32)),
                                   P.ctypes.data_as(C.POINTER(C.c_int32)),
                                   S.ctypes.data_as(C.POINTER(C.c_int32)), len(S), float(eps0),
                                   C.byref(opts), C.byref(h))
    check(st, "dem_build_hierarchy")
    try:
        n = h.n_tris
        out = {
            "tri_verts": np.ctypeslib.as_array(h.tri_verts, (n, 3)).copy(),
            "child_begin": np.ctypeslib.as_array(h.child_begin, (n,)).copy(),
            "child_count": np.ctypeslib.as_array(h.child_count, (n,)).copy(),
            "level_begin": np.ctypeslib.as_array(h.level_begin, (h.n_levels + 1,)).copy(),
            "eps": np.ctypeslib.as_array(h.eps, (n,)).copy(),
            "eps_f32": np.ctypeslib.as_array(h.eps_f32, (n,)).copy(),
            "eps_f64": np.ctypeslib.as_array(h.eps_f64, (n,)).copy(),
            "root_begin": h.root_begin, "root_count": h.root_count,
            "fine_begin": h.fine_begin, "fine_count": h.fine_count, "max_dev": h.max_dev,
        }
    finally:
        lib().dem_hierarchy_free(C.byref(h))
    return out


def build_surrogate_tree(verts: np.ndarray, tris: np.ndarray, **opts) -> dict:
    """dem_build_surrogate_tree on one mesh (k-means splits, Appendix A
    surrogates); ``opts`` override dem_tree_opts fields.  Returns numpy
    copies: verts (mesh then surrogate vertices), tris, parent, level_sizes,
    fine_order and the levels as a list of triangle arrays."""
    V = np.ascontiguousarray(verts, np.float64).reshape(-1, 3)
    T = np.ascontiguousarray(tris, np.int32).reshape(-1, 3)
    o = _abi.TreeOpts()
    lib().dem_default_tree_opts(C.byref(o))
    for k, v in opts.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    t = _abi.SurrogateTree()
    st = lib().dem_build_surrogate_tree(V.ctypes.data_as(C.POINTER(C.c_double)), len(V),
                                        T.ctypes.data_as(C.POINTER(C.c_int32)), len(T), C.byref(o),
                                        C.byref(t))
    check(st, "dem_build_surrogate_tree")
    try:
        n = t.n_tris
        out = {"verts": np.ctypeslib.as_array(t.verts, (t.n_verts, 3)).copy(),
               "tris": np.ctypeslib.as_array(t.tris, (n, 3)).copy(),
               "parent": np.ctypeslib.as_array(t.parent, (n,)).copy(),
               "level_sizes": np.ctypeslib.as_array(t.level_sizes, (t.n_levels,)).copy(),
               "fine_order": np.ctypeslib.as_array(t.fine_order, (len(T),)).copy()}
    finally:
        lib().dem_surrogate_tree_free(C.byref(t))
    offs = np.cumsum([0] + list(out["level_sizes"]))
    out["levels"] = [out["tris"][offs[l]:offs[l + 1]] for l in range(len(offs) - 1)]
    return out


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


# ------------------------------------------------------------------ scene
class DeviceScene:
    """A scene packed into dem_scene's global numbering, resident on the GPU.

    Triangles are numbered particle by particle, coarsest level first; the
    fine triangles of particle p are [fine_begin[p], fine_begin[p]+fine_count[p]).
    ``verts`` is the (3, V) world-coordinate tensor the kernels read; replace
    its contents (same tensor) to move the particles.

    ``lazy`` (default) hands the library the surrogates whose children are
    fine, grouped by depth, so that a step writes fine soup records only for
    the children of surrogates that survived in some pair; ``lazy=False``
    writes every record every step.
    """

    def __init__(self, scene, device="cuda", coord_scale: Optional[float] = None,
                 hier_levels: bool = True, lazy: bool = True, rel_slack: float = 1e-6):
        self.scene = scene
        self.device = torch.device(device)
        self.precision = _abi.DEM_F64 if scene.dtype == "f64" else _abi.DEM_F32
        self.dtype = torch.float64 if scene.dtype == "f64" else torch.float32
        worlds = [scene.world(p) for p in range(len(scene.particles))]
        if coord_scale is None:
            coord_scale = 1.25 * max(float(np.abs(w).max()) for w in worlds) + 1.0
        tv, cb, cc, tp, ep, rb, rc, fb, fc, vb = [], [], [], [], [], [], [], [], [], []
        tpar, tdep = [], []  # parent (global id, -1 for roots) and tree depth of every triangle
        fine_par = {}  # depth -> global ids of surrogates whose children are fine
        nv = nt = 0
        n_levels_max = 1
        self.max_dev = 0.0
        for p, part in enumerate(scene.particles):
            levels = part.levels if hier_levels else [part.levels[-1]]
            sizes = [len(l) for l in levels]
            offs = np.cumsum([0] + sizes)
            tris = np.concatenate(levels).astype(np.int32)
            parent = np.full(len(tris), -1, np.int32)
            if hier_levels:
                absolute = getattr(part, "parents_absolute", False)
                for l in range(1, len(levels)):
                    parent[offs[l]:offs[l + 1]] = part.parents[l] + (0 if absolute else offs[l - 1])
            h = build_hierarchy(worlds[p], tris, parent, sizes, part.eps0, coord_scale, rel_slack)
            depth = np.zeros(len(tris), np.int64)
            for l in range(1, len(levels)):
                depth[offs[l]:offs[l + 1]] = depth[parent[offs[l]:offs[l + 1]]] + 1
            tpar.append(np.where(parent >= 0, parent + nt, -1))
            tdep.append(depth)
            self.max_dev = max(self.max_dev, h["max_dev"])
            n = len(tris)
            tv.append(h["tri_verts"] + nv)
            cb.append(np.where(h["child_count"] > 0, h["child_begin"] + nt, 0))
            cc.append(h["child_count"])
            tp.append(np.full(n, p, np.int32))
            ep.append(h["eps_f64"] if self.precision == _abi.DEM_F64 else h["eps_f32"])
            kids_fine = (h["child_count"] > 0) & (h["child_begin"] >= h["fine_begin"])
            for lev in range(len(levels) - 1):
                ids = np.nonzero(kids_fine[offs[lev]:offs[lev + 1]])[0] + offs[lev] + nt
                if len(ids):
                    fine_par.setdefault(lev, []).append(ids)
            rb.append(nt + h["root_begin"]); rc.append(h["root_count"])
            fb.append(nt + h["fine_begin"]); fc.append(h["fine_count"])
            vb.append(nv)
            n_levels_max = max(n_levels_max, len(levels))
            nv += len(worlds[p])
            nt += n
        d = self.device
        i32 = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.int32), device=d)
        self.n_verts, self.n_tris, self.n_particles = nv, nt, len(scene.particles)
        self.n_levels_max = n_levels_max
        self.vert_begin = np.array(vb, np.int64)
        self.verts_host = np.concatenate(worlds)  # (V,3) f64 (precision-rounded)
        self.verts = torch.as_tensor(self.verts_host.T.copy(), dtype=self.dtype, device=d).contiguous()
        self.tri_verts_host = np.concatenate(tv)
        self.tri_verts = i32(self.tri_verts_host.T.copy())
        self.child_begin = i32(np.concatenate(cb))
        self.child_count = i32(np.concatenate(cc))
        self.tri_particle = i32(np.concatenate(tp))
        self.tri_parent_host = np.concatenate(tpar).astype(np.int32)
        self.tri_depth_host = np.concatenate(tdep).astype(np.uint8)
        self.tri_parent = i32(self.tri_parent_host)
        self.tri_depth = torch.as_tensor(self.tri_depth_host, device=d)
        self.tri_eps = torch.as_tensor(np.concatenate(ep), dtype=self.dtype, device=d)
        self.root_begin, self.root_count = i32(rb), i32(rc)
        self.fine_begin_host = np.array(fb, np.int64)
        self.fine_count_host = np.array(fc, np.int64)
        self.root_count_host = np.array(rc, np.int64)
        self.fine_begin, self.fine_count = i32(fb), i32(fc)
        self.pairs_host = np.asarray(scene.pairs, np.int32).reshape(-1, 2)
        if len(self.pairs_host) and (self.pairs_host.min() < 0 or self.pairs_host.max() >= len(scene.particles)
                                     or np.any(self.pairs_host[:, 0] == self.pairs_host[:, 1])):
            raise DemError("candidate pairs must join two different existing particles")
        self.pairs = i32(self.pairs_host.T.copy())  # (2, P)
        self.coord_scale = coord_scale
        self.pose = None
        self.lazy = lazy and n_levels_max > 1
        groups = [np.concatenate(fine_par[d]) if d in fine_par else np.zeros(0, np.int64)
                  for d in range(n_levels_max)]
        self.fine_parent_begin_host = np.cumsum([0] + [len(g) for g in groups]).astype(np.int64)
        self.fine_parents = i32(np.concatenate(groups) if groups else np.zeros(0)) if self.lazy else None
        # records the flatten kernel writes every step (lazy: surrogates and roots)
        cc_all = np.concatenate(cc)
        n_fine_roots = int(sum(r for r, f in zip(rc, fc) if r == f))
        self.n_eager_records = int(np.sum(cc_all > 0)) + n_fine_roots if self.lazy else nt
        self._refresh()

    def _refresh(self):
        s = _abi.Scene()
        s.precision = self.precision
        s.n_verts, s.n_tris, s.n_particles = self.n_verts, self.n_tris, self.n_particles
        s.n_levels_max = self.n_levels_max
        s.verts = self.verts.data_ptr()
        s.tri_verts = self.tri_verts.data_ptr()
        s.child_begin = self.child_begin.data_ptr()
        s.child_count = self.child_count.data_ptr()
        s.tri_particle = self.tri_particle.data_ptr()
        s.tri_eps = self.tri_eps.data_ptr()
        s.root_begin, s.root_count = self.root_begin.data_ptr(), self.root_count.data_ptr()
        s.fine_begin, s.fine_count = self.fine_begin.data_ptr(), self.fine_count.data_ptr()
        s.pose = None if self.pose is None else self.pose.data_ptr()
        s.tri_parent = self.tri_parent.data_ptr()
        s.tri_depth = self.tri_depth.data_ptr()
        if self.lazy and len(self.fine_parents):
            s.fine_parents = self.fine_parents.data_ptr()
            for d, v in enumerate(self.fine_parent_begin_host):
                s.fine_parent_begin[d] = int(v)
        else:
            s.fine_parents = None
        self.c = s

    def set_verts(self, verts: torch.Tensor):
        """Point the scene at another (3, V) tensor of the scene's dtype."""
        assert verts.shape == (3, self.n_verts) and verts.dtype == self.dtype and verts.is_contiguous()
        self.verts = verts
        self._refresh()

    def set_pose(self, pose: Optional[torch.Tensor]):
        """Per-particle rigid motion (n_particles, 12) = row-major R then c,
        applied in the flatten kernel (world = R v + c); None disables."""
        if pose is not None:
            assert pose.shape == (self.n_particles, 12) and pose.dtype == self.dtype and pose.is_contiguous()
        self.pose = pose
        self._refresh()

    @property
    def n_pairs(self) -> int:
        return len(self.pairs_host)

    def n_fine_pairs(self) -> int:
        F = self.fine_count_host
        return int(np.sum(F[self.pairs_host[:, 0]] * F[self.pairs_host[:, 1]]))


# ------------------------------------------------------------------ calls
def make_params(mode: str = "hier", **kw) -> _abi.Params:
    """Default dem_params with overrides; ``name.index`` sets one element of
    an array field (e.g. ``level_grid.3``)."""
    p = _abi.default_params()
    p.mode = _abi.DEM_MODE_HIER if mode == "hier" else _abi.DEM_MODE_FLAT
    for k, v in kw.items():
        field, _, idx = k.partition(".")
        if not hasattr(p, field):
            raise KeyError(k)
        if idx:
            getattr(p, field)[int(idx)] = v
        else:
            setattr(p, field, v)
    return p


@dataclass
class ContactBuffers:
    capacity: int
    pi: torch.Tensor
    pj: torch.Tensor
    ti: torch.Tensor
    tj: torch.Tensor
    d: torch.Tensor
    x: torch.Tensor
    n: torch.Tensor
    count: torch.Tensor
    adjoint: Optional[torch.Tensor] = None  # [DEM_ADJOINT_ROWS, capacity]: read by the backward

    @staticmethod
    def alloc(capacity: int, dtype, device, adjoint: bool = True) -> "ContactBuffers":
        # a multiple of 4: the backward then reads four contacts' rows per 16-byte load
        cap = max(4, (int(capacity) + 3) // 4 * 4)
        z = lambda *s, dt=torch.int32: torch.zeros(*s, dtype=dt, device=device)
        return ContactBuffers(cap, z(cap), z(cap), z(cap), z(cap), z(cap, dt=dtype), z(3, cap, dt=dtype),
                              z(3, cap, dt=dtype), z(1),
                              z(_abi.DEM_ADJOINT_ROWS, cap, dt=dtype) if adjoint else None)

    def c(self) -> _abi.Contacts:
        s = _abi.Contacts()
        s.capacity = self.capacity
        s.pi, s.pj, s.ti, s.tj = (t.data_ptr() for t in (self.pi, self.pj, self.ti, self.tj))
        s.d, s.x, s.n = self.d.data_ptr(), self.x.data_ptr(), self.n.data_ptr()
        s.count = self.count.data_ptr()
        s.adjoint = self.adjoint.data_ptr() if self.adjoint is not None else None
        return s


class ContactSorter:
    """dem_sort_contacts with its workspace: a contact list of up to
    ``capacity`` entries put in (ti, tj) order, in place, on the current
    stream (graph-capturable)."""

    def __init__(self, ds: "DeviceScene", capacity: int):
        self.ds, self.capacity = ds, int(capacity)
        nbytes = lib().dem_sort_contacts_workspace_bytes(C.byref(ds.c), self.capacity)
        if nbytes == 0:
            raise DemError("dem_sort_contacts_workspace_bytes rejected the scene or capacity")
        self.ws = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=ds.device)
        self.ws_ptr = self.ws.data_ptr() + (-self.ws.data_ptr()) % 256
        self.ws_bytes = int(nbytes)

    def run(self, contacts: "ContactBuffers", status: torch.Tensor):
        assert contacts.capacity <= self.capacity
        cs = contacts.c()
        st = lib().dem_sort_contacts(C.byref(self.ds.c), C.byref(cs), C.c_void_p(self.ws_ptr), self.ws_bytes,
                                     _ptr(status), C.c_void_p(torch.cuda.current_stream(self.ds.device).cuda_stream))
        check(st, "dem_sort_contacts")


class ContactEngine:
    """Preallocated buffers + the C-ABI calls for one scene.

    ``forward()`` enqueues dem_find_contacts (contacts and energy), and with
    ``deterministic`` dem_sort_contacts after it (contacts in (ti, tj) order);
    ``backward()`` dem_contact_backward.  Neither synchronises, so a step can
    be captured in a CUDA/HIP graph; ``check()`` synchronises and raises on
    device-reported overflow.  With ``adjoint`` (default) the contacts carry
    their adjoint rows, and the backward reads them instead of solving each
    pair's closest points again.
    """

    def __init__(self, ds: DeviceScene, params: Optional[_abi.Params] = None,
                 contact_capacity: Optional[int] = None, energy_k: float = 1e4, deterministic: bool = False,
                 adjoint: bool = True):
        self.ds = ds
        self.adjoint = adjoint
        self.deterministic = deterministic
        self.sorter = None
        self.p = params if params is not None else make_params("hier")
        self.p.energy_k = float(energy_k)
        dev = ds.device
        if contact_capacity is None:
            contact_capacity = ds.n_fine_pairs() if self.p.dense_distance else max(1 << 16, 64 * ds.n_pairs)
        if self.p.dense_distance:
            # every fine pair is listed; segments fill unevenly
            self.p.near_capacity = max(int(self.p.near_capacity), int(1.5 * ds.n_fine_pairs()) + 8 * 65536)
        if self.p.mode == _abi.DEM_MODE_FLAT:
            ti, tj = self.p.flat_tile_i, self.p.flat_tile_j
            F = ds.fine_count_host
            a, b = F[ds.pairs_host[:, 0]], F[ds.pairs_host[:, 1]]
            tiles = int(np.sum(((a + ti - 1) // ti) * ((b + tj - 1) // tj)))
            self.p.queue_capacity = max(int(self.p.queue_capacity), 2 * tiles + 8 * 64)
        self.contacts = ContactBuffers.alloc(contact_capacity, ds.dtype, dev, adjoint=adjoint)
        self.stats = torch.zeros(_abi.STATS_WORDS, dtype=torch.int64, device=dev)
        self.status = torch.zeros(1, dtype=torch.int32, device=dev)
        self.energy = torch.zeros(1, dtype=torch.float64, device=dev)
        self.energy_bwd = torch.zeros(1, dtype=torch.float64, device=dev)
        self.generation = 0  # forward() calls so far: the soup and contacts belong to the last one
        self._alloc_ws()

    def _alloc_ws(self):
        nbytes = lib().dem_workspace_bytes(C.byref(self.ds.c), self.ds.n_pairs, C.byref(self.p))
        if nbytes == 0:
            raise DemError("dem_workspace_bytes rejected the scene or parameters")
        self.ws = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=self.ds.device)
        off = (-self.ws.data_ptr()) % 256
        self.ws_ptr = self.ws.data_ptr() + off
        self.ws_bytes = int(nbytes)

    def _stream(self):
        return C.c_void_p(torch.cuda.current_stream(self.ds.device).cuda_stream)

    def forward(self, with_energy: bool = True):
        self.generation += 1
        cs = self.contacts.c()
        st = lib().dem_find_contacts(C.byref(self.ds.c), _ptr(self.ds.pairs), self.ds.n_pairs,
                                     C.byref(self.p), C.byref(cs), C.c_void_p(self.ws_ptr),
                                     self.ws_bytes, _ptr(self.stats), _ptr(self.status),
                                     _ptr(self.energy) if with_energy else None, self._stream())
        check(st, "dem_find_contacts")
        if self.deterministic:
            if self.sorter is None or self.sorter.capacity < self.contacts.capacity:
                self.sorter = ContactSorter(self.ds, self.contacts.capacity)
            self.sorter.run(self.contacts, self.status)

    def backward(self, grad_verts: torch.Tensor, grad_E: Optional[torch.Tensor] = None,
                 energy: bool = False):
        assert grad_verts.shape == (3, self.ds.n_verts) and grad_verts.dtype == self.ds.dtype
        cs = self.contacts.c()
        st = lib().dem_contact_backward(C.byref(self.ds.c), C.byref(cs), float(self.p.energy_k),
                                        _ptr(grad_E), _ptr(grad_verts),
                                        _ptr(self.energy_bwd) if energy else None,
                                        C.c_void_p(self.ws_ptr), self.ws_bytes, _ptr(self.status),
                                        self._stream())
        check(st, "dem_contact_backward")

    # ---------------------------------------------------------- host-side reads
    def counters(self) -> dict:
        """Segment fills of the level queues, near list and fallback list
        (host copy; layout of the library's counter block)."""
        nseg, L = 8, _abi.DEM_MAX_LEVELS + 1
        nw = L * nseg + 2 * nseg
        off = self.ws_ptr - self.ws.data_ptr()
        w = self.ws[off:off + 4 * nw].view(torch.int32).cpu().numpy().astype(np.int64) & 0xFFFFFFFF
        return {"tail": w[:L * nseg].reshape(L, nseg), "near": w[L * nseg:L * nseg + nseg],
                "fb": w[L * nseg + nseg:]}

    def check(self) -> int:
        torch.cuda.synchronize(self.ds.device)
        return int(self.status.item()) & 0xFFFFFFFF

    def count(self) -> int:
        return int(self.contacts.count.item()) & 0xFFFFFFFF

    def run(self, with_energy: bool = True, max_retries: int = 6):
        """forward() + synchronise; grows capacities and reruns on overflow."""
        for _ in range(max_retries):
            self.forward(with_energy)
            status = self.check()
            if status & _abi.DEM_DEV_NONFINITE:
                raise DemError("non-finite coordinates or distances")
            if status & _abi.DEM_DEV_BAD_TREE:
                raise DemError("malformed surrogate tree (child counts)")
            if status & _abi.DEM_DEV_STALLED:
                # the persistent descent's grid could not synchronise (e.g. not
                # all of its blocks were resident): one launch per depth instead
                self.p.persistent = 0
                continue
            if not status & (_abi.DEM_DEV_CONTACT_OVERFLOW | _abi.DEM_DEV_QUEUE_OVERFLOW |
                             _abi.DEM_DEV_NEAR_OVERFLOW):
                return status
            ctr = self.counters()
            if status & _abi.DEM_DEV_CONTACT_OVERFLOW:
                self.contacts = ContactBuffers.alloc(int(self.count() * 1.25) + 1024, self.ds.dtype,
                                                     self.ds.device, adjoint=self.adjoint)
            grow = False
            # lists are split into 8 segments: size for the fullest one
            if status & _abi.DEM_DEV_QUEUE_OVERFLOW:
                need = 8 * int(ctr["tail"].max())
                self.p.queue_capacity = max(2 * self.p.queue_capacity, int(1.25 * need) + 1024)
                grow = True
            if status & _abi.DEM_DEV_NEAR_OVERFLOW:
                need = 8 * int(max(ctr["near"].max(), ctr["fb"].max()))
                self.p.near_capacity = max(2 * self.p.near_capacity, int(1.25 * need) + 1024)
                grow = True
            if grow:
                self.ws = None
                self._alloc_ws()
        raise DemError("capacities kept overflowing")

    def stats_dict(self) -> dict:
        return _stats_dict(self.stats)

    def result(self) -> dict:
        """Host copy of the contacts (after run())."""
        n = min(self.count(), self.contacts.capacity)
        c = self.contacts
        return {"pi": c.pi[:n].cpu().numpy(), "pj": c.pj[:n].cpu().numpy(),
                "ti": c.ti[:n].cpu().numpy(), "tj": c.tj[:n].cpu().numpy(),
                "d": c.d[:n].double().cpu().numpy(), "x": c.x[:, :n].double().cpu().numpy().T,
                "n": c.n[:, :n].double().cpu().numpy().T, "energy": float(self.energy.item())}


def _stats_dict(stats: torch.Tensor) -> dict:
    s = stats.cpu().numpy().view(np.uint64)
    L = _abi.DEM_MAX_LEVELS
    return {"evals": s[0:L].astype(np.int64), "survivors": s[L:2 * L].astype(np.int64),
            "near": int(s[2 * L]), "certified": int(s[2 * L + 1]), "fallback": int(s[2 * L + 2]),
            "contacts": int(s[2 * L + 3]), "items": s[2 * L + 4:3 * L + 4].astype(np.int64),
            "frontier_leaves": int(s[3 * L + 4]), "frontier_unfolded": int(s[3 * L + 5]),
            "frontier_collapsed": int(s[3 * L + 6]), "fine_records": int(s[3 * L + 7])}


class FrontierEngine:
    """Persistent active sets for one scene: dem_frontier_init once, then
    dem_frontier_step per Picard iteration or time step (Algorithm 6).

    Buffers (two leaf buffers, the device state word, the memory set, the
    contacts and the workspace) are allocated here with torch; ``step()``
    enqueues one call on the current stream without synchronising.
    """

    def __init__(self, ds: DeviceScene, params: Optional[_abi.Params] = None,
                 capacity: Optional[int] = None, memory_capacity: Optional[int] = None,
                 contact_capacity: Optional[int] = None, energy_k: float = 1e4, adjoint: bool = True):
        self.ds = ds
        self.adjoint = adjoint
        self.p = params if params is not None else make_params("hier")
        self.p.energy_k = float(energy_k)
        dev = ds.device
        rc = ds.root_count_host
        P = ds.pairs_host
        self.n_roots = int(np.sum(rc[P[:, 0]] * rc[P[:, 1]])) if len(P) else 0
        cap = int(capacity) if capacity is not None else max(1 << 16, 64 * self.n_roots)
        mem = int(memory_capacity) if memory_capacity is not None else max(1 << 12, cap // 2)
        self.memory_capacity = 1 << (max(64, mem) - 1).bit_length()
        self.memory = torch.empty(self.memory_capacity, dtype=torch.int64, device=dev)
        self.state = torch.zeros(4, dtype=torch.int32, device=dev)
        self._alloc_leaves(cap)
        if contact_capacity is None:
            contact_capacity = max(1 << 16, 64 * ds.n_pairs)
        self.contacts = ContactBuffers.alloc(contact_capacity, ds.dtype, dev, adjoint=adjoint)
        self.stats = torch.zeros(_abi.STATS_WORDS, dtype=torch.int64, device=dev)
        self.status = torch.zeros(1, dtype=torch.int32, device=dev)
        self.energy = torch.zeros(1, dtype=torch.float64, device=dev)
        self.energy_bwd = torch.zeros(1, dtype=torch.float64, device=dev)
        self._alloc_ws()

    def _alloc_leaves(self, cap: int):
        self.capacity = int(cap)
        self.leaf_bufs = [torch.zeros(self.capacity, 4, dtype=torch.int32, device=self.ds.device)
                          for _ in range(2)]

    def _alloc_ws(self):
        nbytes = lib().dem_frontier_workspace_bytes(C.byref(self.ds.c), self.ds.n_pairs, C.byref(self.p),
                                                    self.capacity)
        if nbytes == 0:
            raise DemError("dem_frontier_workspace_bytes rejected the scene or parameters")
        self.ws = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=self.ds.device)
        off = (-self.ws.data_ptr()) % 256
        self.ws_ptr = self.ws.data_ptr() + off
        self.ws_bytes = int(nbytes)

    def c(self) -> _abi.Frontier:
        f = _abi.Frontier()
        f.capacity = self.capacity
        f.leaves[0] = self.leaf_bufs[0].data_ptr()
        f.leaves[1] = self.leaf_bufs[1].data_ptr()
        f.state = self.state.data_ptr()
        f.memory_capacity = self.memory_capacity
        f.memory = self.memory.data_ptr()
        return f

    def _stream(self):
        return C.c_void_p(torch.cuda.current_stream(self.ds.device).cuda_stream)

    def init(self):
        f = self.c()
        st = lib().dem_frontier_init(C.byref(self.ds.c), _ptr(self.ds.pairs), self.ds.n_pairs, C.byref(self.p),
                                     C.byref(f), C.c_void_p(self.ws_ptr), self.ws_bytes, _ptr(self.status),
                                     self._stream())
        check(st, "dem_frontier_init")
        if self.check() & _abi.DEM_DEV_FRONTIER_OVERFLOW:
            need = int(self.state_host()[2])
            self._alloc_leaves(max(2 * self.capacity, int(1.25 * need) + 1024))
            self._alloc_ws()
            return self.init()

    def step(self, with_energy: bool = True):
        f = self.c()
        cs = self.contacts.c()
        st = lib().dem_frontier_step(C.byref(self.ds.c), C.byref(self.p), C.byref(f), C.byref(cs),
                                     C.c_void_p(self.ws_ptr), self.ws_bytes, _ptr(self.stats), _ptr(self.status),
                                     _ptr(self.energy) if with_energy else None, self._stream())
        check(st, "dem_frontier_step")

    def backward(self, grad_verts: torch.Tensor, grad_E: Optional[torch.Tensor] = None, energy: bool = False):
        """dem_contact_backward on the last step's contacts."""
        assert grad_verts.shape == (3, self.ds.n_verts) and grad_verts.dtype == self.ds.dtype
        cs = self.contacts.c()
        st = lib().dem_contact_backward(C.byref(self.ds.c), C.byref(cs), float(self.p.energy_k),
                                        _ptr(grad_E), _ptr(grad_verts),
                                        _ptr(self.energy_bwd) if energy else None,
                                        C.c_void_p(self.ws_ptr), self.ws_bytes, _ptr(self.status),
                                        self._stream())
        check(st, "dem_contact_backward")

    # ---------------------------------------------------------- host-side reads
    def check(self) -> int:
        torch.cuda.synchronize(self.ds.device)
        return int(self.status.item()) & 0xFFFFFFFF

    def state_host(self) -> np.ndarray:
        return self.state.cpu().numpy().astype(np.int64) & 0xFFFFFFFF

    def leaves(self) -> np.ndarray:
        """(n, 4) int64 leaf records {t_i, t_j, flags, info} of the current sets."""
        cur, n = (int(v) for v in self.state_host()[:2])
        return self.leaf_bufs[cur][:n].cpu().numpy().astype(np.int64) & 0xFFFFFFFF

    def count(self) -> int:
        return int(self.contacts.count.item()) & 0xFFFFFFFF

    def run_step(self, with_energy: bool = True, max_retries: int = 6) -> int:
        """step() + synchronise; on overflow the sets are unchanged, so the
        capacities grow and the same step runs again."""
        for _ in range(max_retries):
            self.step(with_energy)
            status = self.check()
            if status & _abi.DEM_DEV_NONFINITE:
                raise DemError("non-finite coordinates or distances")
            if status & _abi.DEM_DEV_BAD_TREE:
                raise DemError("malformed surrogate tree (child counts)")
            over = (_abi.DEM_DEV_CONTACT_OVERFLOW | _abi.DEM_DEV_NEAR_OVERFLOW | _abi.DEM_DEV_FRONTIER_OVERFLOW)
            if not status & over:
                return status
            if status & _abi.DEM_DEV_CONTACT_OVERFLOW:
                self.contacts = ContactBuffers.alloc(int(self.count() * 1.25) + 1024, self.ds.dtype, self.ds.device,
                                                     adjoint=self.adjoint)
            if status & _abi.DEM_DEV_NEAR_OVERFLOW:
                self.p.near_capacity = 2 * int(self.p.near_capacity)
            if status & _abi.DEM_DEV_FRONTIER_OVERFLOW:
                need = int(self.state_host()[2])
                if need <= self.capacity:
                    raise DemError("frontier memory set is full: initialise again with a larger memory_capacity")
                self.reserve(max(2 * self.capacity, int(1.25 * need) + 1024))
            self.ws = None
            self._alloc_ws()
        raise DemError("capacities kept overflowing")

    def reserve(self, capacity: int):
        """Grow both leaf buffers to ``capacity`` keeping the current sets
        (and the memory set); synchronises."""
        if capacity <= self.capacity:
            return
        old = self.leaves()
        self._alloc_leaves(int(capacity))
        self.leaf_bufs[0][:len(old)] = torch.as_tensor(old.astype(np.uint32).view(np.int32), device=self.ds.device)
        self.state.copy_(torch.tensor([0, len(old), len(old), 0], dtype=torch.int32))
        self.ws = None
        self._alloc_ws()

    def run_to_fixed_point(self, max_steps: int = 64) -> int:
        """run_step() at the current positions until a step neither widens
        nor narrows; returns the number of steps."""
        for k in range(1, max_steps + 1):
            self.run_step()
            s = self.stats_dict()
            if s["frontier_unfolded"] == 0 and s["frontier_collapsed"] == 0:
                return k
        raise DemError("active sets kept changing")

    def stats_dict(self) -> dict:
        return _stats_dict(self.stats)

    def result(self) -> dict:
        n = min(self.count(), self.contacts.capacity)
        c = self.contacts
        return {"pi": c.pi[:n].cpu().numpy(), "pj": c.pj[:n].cpu().numpy(),
                "ti": c.ti[:n].cpu().numpy(), "tj": c.tj[:n].cpu().numpy(),
                "d": c.d[:n].double().cpu().numpy(), "energy": float(self.energy.item())}


@dataclass
class MergedBuffers:
    capacity: int
    pi: torch.Tensor
    pj: torch.Tensor
    x: torch.Tensor
    n: torch.Tensor
    f: torch.Tensor
    members: torch.Tensor
    count: torch.Tensor

    @staticmethod
    def alloc(capacity: int, dtype, device) -> "MergedBuffers":
        cap = max(1, int(capacity))
        z = lambda *s, dt=torch.int32: torch.zeros(*s, dtype=dt, device=device)
        return MergedBuffers(cap, z(cap), z(cap), z(3, cap, dt=dtype), z(3, cap, dt=dtype), z(3, cap, dt=dtype),
                             z(cap), z(1))

    def c(self) -> _abi.Merged:
        m = _abi.Merged()
        m.capacity = self.capacity
        m.pi, m.pj, m.x, m.n, m.f, m.members, m.count = (
            t.data_ptr() for t in (self.pi, self.pj, self.x, self.n, self.f, self.members, self.count))
        return m


class ForceEngine:
    """dem_contact_forces for one scene: merged contact points, their forces
    and per-particle force and torque, from a contact list of up to
    ``contact_capacity`` entries (the output of ContactEngine or
    FrontierEngine)."""

    def __init__(self, ds: DeviceScene, contact_capacity: int, merged_capacity: Optional[int] = None):
        self.ds = ds
        dev = ds.device
        self.contact_capacity = int(contact_capacity)
        nbytes = lib().dem_contact_forces_workspace_bytes(self.contact_capacity)
        if nbytes == 0:
            raise DemError("dem_contact_forces_workspace_bytes rejected the capacity")
        self.ws = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=dev)
        self.ws_ptr = self.ws.data_ptr() + (-self.ws.data_ptr()) % 256
        self.ws_bytes = int(nbytes)
        self.merged = MergedBuffers.alloc(merged_capacity or self.contact_capacity, ds.dtype, dev)
        self.group = torch.zeros(max(1, self.contact_capacity), dtype=torch.int32, device=dev)
        self.force = torch.zeros(3, ds.n_particles, dtype=ds.dtype, device=dev)
        self.torque = torch.zeros(3, ds.n_particles, dtype=ds.dtype, device=dev)
        self.status = torch.zeros(1, dtype=torch.int32, device=dev)

    def run(self, contacts: ContactBuffers, mass: torch.Tensor, centre: torch.Tensor, k_s: float = 1000.0,
            merge_scale: float = 1.0, with_group: bool = True):
        """Enqueue: force and torque are zeroed, then accumulated."""
        assert contacts.capacity <= self.contact_capacity
        assert mass.shape == (self.ds.n_particles,) and mass.dtype == self.ds.dtype and mass.is_contiguous()
        assert centre.shape == (3, self.ds.n_particles) and centre.dtype == self.ds.dtype and centre.is_contiguous()
        self.force.zero_()
        self.torque.zero_()
        self.status.zero_()
        cs = contacts.c()
        mc = self.merged.c()
        st = lib().dem_contact_forces(C.byref(self.ds.c), C.byref(cs), _ptr(mass), _ptr(centre), float(k_s),
                                      float(merge_scale), C.byref(mc), _ptr(self.group) if with_group else None,
                                      _ptr(self.force), _ptr(self.torque), C.c_void_p(self.ws_ptr), self.ws_bytes,
                                      _ptr(self.status), C.c_void_p(torch.cuda.current_stream(self.ds.device).cuda_stream))
        check(st, "dem_contact_forces")

    def check(self) -> int:
        torch.cuda.synchronize(self.ds.device)
        return int(self.status.item()) & 0xFFFFFFFF

    def result(self, n_contacts: int) -> dict:
        m = self.merged
        k = min(int(m.count.item()) & 0xFFFFFFFF, m.capacity)
        return {"pi": m.pi[:k].cpu().numpy(), "pj": m.pj[:k].cpu().numpy(),
                "x": m.x[:, :k].double().cpu().numpy().T, "n": m.n[:, :k].double().cpu().numpy().T,
                "f": m.f[:, :k].double().cpu().numpy().T, "members": m.members[:k].cpu().numpy(),
                "group": self.group[:n_contacts].cpu().numpy(),
                "force": self.force.double().cpu().numpy().T, "torque": self.torque.double().cpu().numpy().T}


class DemContactEnergy(torch.autograd.Function):
    """E(verts) = k * sum over contacts of max(0, eps_i + eps_j - d)^2.

    forward: dem_find_contacts (contacts + energy); backward: the adjoint
    kernel dem_contact_backward, which recomputes the closest points.
    """

    @staticmethod
    def forward(ctx, verts: torch.Tensor, engine: ContactEngine):
        if verts.data_ptr() != engine.ds.verts.data_ptr():
            engine.ds.set_verts(verts.detach().contiguous())
        # run(): synchronises, grows the buffers and repeats the call on any
        # overflow, and raises on non-finite input, so that the energy and
        # the contact list the backward differentiates are complete
        engine.run(with_energy=True)
        ctx.engine = engine
        ctx.generation = engine.generation
        return engine.energy[0].to(verts.dtype).clone()

    @staticmethod
    def backward(ctx, grad_E: torch.Tensor):
        eng = ctx.engine
        if eng.generation != ctx.generation:
            raise DemError("the engine ran another forward since this energy was computed; its contacts and "
                           "soup now belong to that call (use one engine per pending backward)")
        g = torch.zeros(3, eng.ds.n_verts, dtype=eng.ds.dtype, device=eng.ds.device)
        gE = grad_E.detach().to(torch.float64).reshape(1).contiguous()
        eng.backward(g, gE)
        return g, None


def contact_energy(verts: torch.Tensor, engine: ContactEngine) -> torch.Tensor:
    return DemContactEnergy.apply(verts, engine)
