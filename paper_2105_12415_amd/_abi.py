"""ctypes view of include/dem.h and the loader of libdem.so.

Argument marshalling only: every computation of the path runs in the HIP
kernels behind these symbols.  Importing this module fails loudly when the
library has not been built; there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# DEM_LIBRARY selects another build of the same ABI (e.g. a tuning variant).
LIB_PATH = os.environ.get("DEM_LIBRARY") or os.path.join(HERE, "libdem.so")

DEM_OK, DEM_ERR_ARG, DEM_ERR_CAPACITY, DEM_ERR_HIP, DEM_ERR_NOT_CONSERVATIVE, DEM_ERR_OOM = 0, -1, -2, -3, -4, -5
DEM_F32, DEM_F64 = 0, 1
DEM_MODE_FLAT, DEM_MODE_HIER = 0, 1
DEM_DEV_CONTACT_OVERFLOW = 0x1
DEM_DEV_QUEUE_OVERFLOW = 0x2
DEM_DEV_NEAR_OVERFLOW = 0x4
DEM_DEV_NONFINITE = 0x8
DEM_DEV_BAD_TREE = 0x10
DEM_DEV_FRONTIER_OVERFLOW = 0x20
DEM_DEV_STALLED = 0x40
DEM_ADJOINT_ROWS = 9
DEM_MAX_LEVELS = 32
DEM_MAX_CHILDREN = 16
DEM_SCRATCH_BYTES = 64 << 20

# Every exported symbol declared in include/dem.h.
EXPORTS = ("dem_build_hierarchy", "dem_hierarchy_free", "dem_default_params", "dem_workspace_bytes",
           "dem_find_contacts", "dem_contact_backward", "dem_status_string", "dem_version",
           "dem_default_tree_opts", "dem_build_surrogate_tree", "dem_surrogate_tree_free",
           "dem_frontier_workspace_bytes", "dem_frontier_init", "dem_frontier_step",
           "dem_contact_forces_workspace_bytes", "dem_contact_forces",
           "dem_sort_contacts_workspace_bytes", "dem_sort_contacts", "dem_find_contacts_noalloc")


class BuildOpts(C.Structure):
    _fields_ = [("coord_scale", C.c_double), ("rel_slack", C.c_double)]


class TreeOpts(C.Structure):
    _fields_ = [("fanout", C.c_int32), ("kmeans_iters", C.c_int32), ("fit_iters", C.c_int32),
                ("beta_size", C.c_double), ("alpha_area", C.c_double), ("alpha_inside", C.c_double),
                ("beta_normal", C.c_double)]


class SurrogateTree(C.Structure):
    _fields_ = [("n_verts", C.c_int32), ("verts", C.POINTER(C.c_double)), ("n_tris", C.c_int32),
                ("tris", C.POINTER(C.c_int32)), ("parent", C.POINTER(C.c_int32)), ("n_levels", C.c_int32),
                ("level_sizes", C.POINTER(C.c_int32)), ("fine_order", C.POINTER(C.c_int32))]


class Hierarchy(C.Structure):
    _fields_ = [("n_tris", C.c_int32), ("n_levels", C.c_int32),
                ("tri_verts", C.POINTER(C.c_int32)), ("child_begin", C.POINTER(C.c_int32)),
                ("child_count", C.POINTER(C.c_int32)), ("level_begin", C.POINTER(C.c_int32)),
                ("eps", C.POINTER(C.c_double)), ("eps_f32", C.POINTER(C.c_float)),
                ("eps_f64", C.POINTER(C.c_double)),
                ("root_begin", C.c_int32), ("root_count", C.c_int32),
                ("fine_begin", C.c_int32), ("fine_count", C.c_int32), ("max_dev", C.c_double)]


class Scene(C.Structure):
    _fields_ = [("precision", C.c_int32), ("n_verts", C.c_int32), ("n_tris", C.c_int32),
                ("n_particles", C.c_int32), ("n_levels_max", C.c_int32),
                ("verts", C.c_void_p), ("tri_verts", C.c_void_p), ("child_begin", C.c_void_p),
                ("child_count", C.c_void_p), ("tri_particle", C.c_void_p), ("tri_eps", C.c_void_p),
                ("root_begin", C.c_void_p), ("root_count", C.c_void_p),
                ("fine_begin", C.c_void_p), ("fine_count", C.c_void_p), ("pose", C.c_void_p),
                ("fine_parents", C.c_void_p), ("fine_parent_begin", C.c_int32 * (DEM_MAX_LEVELS + 1)),
                ("tri_parent", C.c_void_p), ("tri_depth", C.c_void_p)]


class Params(C.Structure):
    _fields_ = [("mode", C.c_int32), ("n_iter", C.c_int32), ("omega", C.c_float),
                ("alpha_reg_rel", C.c_float), ("alpha_it_ratio", C.c_float),
                ("init_centroid", C.c_int32), ("dense_distance", C.c_int32), ("certify", C.c_int32),
                ("prune_exact", C.c_int32), ("energy_k", C.c_double), ("block", C.c_int32), ("grid", C.c_int32),
                ("batch_items", C.c_int32), ("flat_tile_i", C.c_int32), ("flat_tile_j", C.c_int32),
                ("seed_chunk", C.c_int32), ("frontier_grid", C.c_int32), ("half_depths", C.c_int32),
                ("level_grid", C.c_int32 * DEM_MAX_LEVELS), ("level_batch", C.c_int32 * DEM_MAX_LEVELS),
                ("queue_capacity", C.c_int64), ("near_capacity", C.c_int64),
                ("events", C.POINTER(C.c_void_p)), ("n_events", C.c_int32),
                ("persistent", C.c_int32), ("persistent_spins", C.c_int32)]


class Contacts(C.Structure):
    _fields_ = [("capacity", C.c_int64), ("pi", C.c_void_p), ("pj", C.c_void_p), ("ti", C.c_void_p),
                ("tj", C.c_void_p), ("d", C.c_void_p), ("x", C.c_void_p), ("n", C.c_void_p),
                ("count", C.c_void_p), ("adjoint", C.c_void_p)]


class Stats(C.Structure):
    _fields_ = [("evals", C.c_uint64 * DEM_MAX_LEVELS), ("survivors", C.c_uint64 * DEM_MAX_LEVELS),
                ("near", C.c_uint64), ("certified", C.c_uint64), ("fallback", C.c_uint64),
                ("contacts", C.c_uint64), ("items", C.c_uint64 * DEM_MAX_LEVELS),
                ("frontier_leaves", C.c_uint64), ("frontier_unfolded", C.c_uint64),
                ("frontier_collapsed", C.c_uint64), ("fine_records", C.c_uint64)]


class Merged(C.Structure):
    _fields_ = [("capacity", C.c_int64), ("pi", C.c_void_p), ("pj", C.c_void_p), ("x", C.c_void_p),
                ("n", C.c_void_p), ("f", C.c_void_p), ("members", C.c_void_p), ("count", C.c_void_p)]


class Frontier(C.Structure):
    _fields_ = [("capacity", C.c_int64), ("leaves", C.c_void_p * 2), ("state", C.c_void_p),
                ("memory_capacity", C.c_int64), ("memory", C.c_void_p)]


STATS_WORDS = C.sizeof(Stats) // 8

_lib = None


class DemError(RuntimeError):
    pass


def lib():
    """Load libdem.so (built by paper_2105_12415_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise DemError(f"{LIB_PATH} is missing: build it with `python -m paper_2105_12415_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.dem_build_hierarchy.argtypes = [C.POINTER(C.c_double), C.c_int32, C.POINTER(C.c_int32),
                                          C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.c_int32,
                                          C.c_double, C.POINTER(BuildOpts), C.POINTER(Hierarchy)]
        L.dem_build_hierarchy.restype = C.c_int
        L.dem_hierarchy_free.argtypes = [C.POINTER(Hierarchy)]
        L.dem_hierarchy_free.restype = None
        L.dem_default_tree_opts.argtypes = [C.POINTER(TreeOpts)]
        L.dem_default_tree_opts.restype = None
        L.dem_build_surrogate_tree.argtypes = [C.POINTER(C.c_double), C.c_int32, C.POINTER(C.c_int32),
                                               C.c_int32, C.POINTER(TreeOpts), C.POINTER(SurrogateTree)]
        L.dem_build_surrogate_tree.restype = C.c_int
        L.dem_surrogate_tree_free.argtypes = [C.POINTER(SurrogateTree)]
        L.dem_surrogate_tree_free.restype = None
        L.dem_default_params.argtypes = [C.POINTER(Params)]
        L.dem_default_params.restype = None
        L.dem_workspace_bytes.argtypes = [C.POINTER(Scene), C.c_int32, C.POINTER(Params)]
        L.dem_workspace_bytes.restype = C.c_size_t
        L.dem_find_contacts.argtypes = [C.POINTER(Scene), vp, C.c_int32, C.POINTER(Params),
                                        C.POINTER(Contacts), vp, C.c_size_t, vp, vp, vp, vp]
        L.dem_find_contacts.restype = C.c_int
        L.dem_find_contacts_noalloc.argtypes = [C.POINTER(Scene), vp, C.c_int32, C.POINTER(Params),
                                                C.POINTER(Contacts), vp, vp, vp, vp]
        L.dem_find_contacts_noalloc.restype = C.c_int
        L.dem_sort_contacts_workspace_bytes.argtypes = [C.POINTER(Scene), C.c_int64]
        L.dem_sort_contacts_workspace_bytes.restype = C.c_size_t
        L.dem_sort_contacts.argtypes = [C.POINTER(Scene), C.POINTER(Contacts), vp, C.c_size_t, vp, vp]
        L.dem_sort_contacts.restype = C.c_int
        L.dem_contact_backward.argtypes = [C.POINTER(Scene), C.POINTER(Contacts), C.c_double, vp, vp,
                                           vp, vp, C.c_size_t, vp, vp]
        L.dem_contact_backward.restype = C.c_int
        L.dem_frontier_workspace_bytes.argtypes = [C.POINTER(Scene), C.c_int32, C.POINTER(Params), C.c_int64]
        L.dem_frontier_workspace_bytes.restype = C.c_size_t
        L.dem_frontier_init.argtypes = [C.POINTER(Scene), vp, C.c_int32, C.POINTER(Params), C.POINTER(Frontier),
                                        vp, C.c_size_t, vp, vp]
        L.dem_frontier_init.restype = C.c_int
        L.dem_frontier_step.argtypes = [C.POINTER(Scene), C.POINTER(Params), C.POINTER(Frontier),
                                        C.POINTER(Contacts), vp, C.c_size_t, vp, vp, vp, vp]
        L.dem_frontier_step.restype = C.c_int
        L.dem_contact_forces_workspace_bytes.argtypes = [C.c_int64]
        L.dem_contact_forces_workspace_bytes.restype = C.c_size_t
        L.dem_contact_forces.argtypes = [C.POINTER(Scene), C.POINTER(Contacts), vp, vp, C.c_double, C.c_double,
                                         C.POINTER(Merged), vp, vp, vp, vp, C.c_size_t, vp, vp]
        L.dem_contact_forces.restype = C.c_int
        L.dem_status_string.argtypes = [C.c_int]
        L.dem_status_string.restype = C.c_char_p
        L.dem_version.argtypes = []
        L.dem_version.restype = C.c_char_p
        _lib = L
    return _lib


def check(status: int, what: str):
    if status != DEM_OK:
        msg = lib().dem_status_string(status).decode()
        raise DemError(f"{what} failed: {msg} ({status})")


def default_params() -> Params:
    p = Params()
    lib().dem_default_params(C.byref(p))
    return p
