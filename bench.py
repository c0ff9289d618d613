#!/usr/bin/env python3
"""Benchmark of the multiresolution contact-detection path on one MI355X.

Default workload (``--workload lattice_fwd_bwd``): the 1000-sphere lattice
(subdivision 3-5, radii log-uniform in [0.5, 2], gaps U(0, 0.1); FP32),
forward + backward of the penalty contact energy k * sum max(0, delta - d)^2,
k = 1e4, with a seeded rigid perturbation of every particle per step; K
steps are captured in one HIP graph and replayed.  Forward-only workloads:
two_spheres_s3_f64, two_spheres_s5, lattice, big_small.

One JSON line is printed: tri-pair evaluations per second of the
hierarchical step (``value``), its ms per step, the plain all-pairs (flat)
step on the same scene for comparison, the roofline of the dominant kernel
(measured with HIP events recorded by the library around each launch), and
the FP64 CPU oracle's rate on a bounded sample of candidate pairs.
"""
from __future__ import annotations

import argparse
import ctypes as C
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "tri-pair evals/s and contact fwd+bwd ms/step: hierarchical batched vs plain all-pairs"
PEAK_FP32_VALU_TFLOPS = 157.3  # 256 CU x 128 FP32 FMA lanes/clk x 2 flop x 2.4 GHz
PEAK_FP64_VALU_TFLOPS = 78.6   # 256 CU x 64 FP64 FMA lanes/clk x 2 flop x 2.4 GHz
PEAK_HBM_GBS = 8000.0


def flops_per_eval(n_iter: int) -> int:
    """Algorithmic floating-point operations of one iterate-and-bound
    evaluation, counted from its formulas (FMA = 2; add, mul, min, max,
    compare, rsqrt = 1; sign changes, absolute values and selects = 0): 74 per
    Newton iteration (residual 24, gradient 20, diagonal step 8, two penalty
    half-steps 22; the first starts at (a, b) = 0 where the residual is the
    vertex difference itself, 24 fewer), plus 3 for the vertex difference, 8
    for clamping the four parameters, 63 for the bound along the direction
    between the two points (residual 24, its length 5, five dot products 25,
    the two support functions 4, combination and normalisation 5) and 10 for
    the rounding slack, the threshold and the test."""
    if n_iter == 0:
        return 84
    return 74 * n_iter - 24 + 84


def exact_pair_flops() -> int:
    """Algorithmic floating-point operations of the exact comparison-based
    distance of one triangle pair and its contact emission (same convention
    as flops_per_eval; a dot product 5, a cross product 9, a 3-vector add 3,
    an FMA on 3-vectors 6): vertices and edges of both triangles 18; normals
    and their squared lengths 28; heights of each triangle's vertices over
    the other's plane 48; the six edge-through-triangle crossing tests
    2 x 157 (three in-plane edge normals 27, per edge the straddle tests 6,
    the plane point 10, three inside tests 27); the six vertex-interior
    candidates 2 x 89 (reciprocal and in-plane gradients 20, per vertex 23);
    squared edge lengths and reciprocals 42; nine segment-segment distances
    with the running minimum 9 x 85; the winner's closest points 30; weights
    4; the square root 1; contact point, normal and adjoint rows 24."""
    return 18 + 28 + 48 + 2 * 157 + 2 * 89 + 42 + 9 * 85 + 30 + 4 + 1 + 24


FLATTEN_BYTES_PER_TRI = 12 + 16 + 64  # indices, per-triangle static data, soup record
FLATTEN_BYTES_SKIPPED = 8             # child count and particle of a triangle left to the lazy pass
FLATTEN_BYTES_PER_VERT = 12


WORKLOADS = {
    "two_spheres_s3_f64": ("two bumped unit spheres, subdivision 3 (1280 tris each), FP64, single level", False),
    "two_spheres_s5": ("two bumped unit spheres, subdivision 5 (20480 tris each), levels s=3/4/5, FP32", False),
    "lattice": ("1000 bumped spheres on a 10x10x10 lattice, subdivision 3-5, radii logU[0.5,2], "
                "gaps U(0,0.1), full icosphere cascades, FP32", False),
    "lattice_fwd_bwd": ("1000 bumped spheres on a 10x10x10 lattice, subdivision 3-5, radii logU[0.5,2], "
                        "gaps U(0,0.1), full icosphere cascades, FP32", True),
    "big_small": ("bumped sphere R=20 subdivision 7 (327680 tris) + 2000 R=0.5 subdivision-3 spheres "
                  "on its surface, FP32", False),
    "lattice_forces": ("1000 bumped spheres on a 10x10x10 lattice, subdivision 3-5, radii logU[0.5,2], "
                       "gaps U(0,0.1), full icosphere cascades, FP32; contact forces: points closer than eps "
                       "merged, force law K_s = 1000, per-particle force and torque (dem_contact_forces)", False),
    "lattice_frontier": ("1000 bumped spheres on a 10x10x10 lattice, subdivision 3-5, radii logU[0.5,2], "
                         "gaps U(0,0.1), full icosphere cascades, FP32; persistent active sets "
                         "(dem_frontier_step, one level of widening / narrowing per step)", True),
}


def step_roofline(ms_step: float, kernels: dict, st: dict, n_pairs: int, n_iter: int, fp64: bool,
                  flat_bytes: float, touched_verts: int, peaks: dict = None) -> dict:
    """Every kernel of the step against the roof that binds it, weighted by
    its time: ALU-bound kernels (the descent, the exact pass) by their
    algorithmic flops against the VALU peak, memory-bound ones (flatten,
    seeding, lazy flattening, backward) by their algorithmic HBM bytes
    against 8 TB/s.  weighted_frac = sum of ms x frac over the step's
    milliseconds (time outside these kernels counts as 0).  Per-unit
    figures: flatten as reported in ``kernels``; seeding 16 B per root item
    written + 24 B per candidate pair read; lazy flattening 92 B per record
    written; the backward 32 + 10 s bytes per contact (its triangle pair
    8 B, its distance and nine adjoint rows of s-byte values, six vertex ids
    24 B) + 6 s bytes per distinct vertex touched (gradient read and
    written)."""
    sz = 8 if fp64 else 4
    peak_alu = PEAK_FP64_VALU_TFLOPS if fp64 else PEAK_FP32_VALU_TFLOPS
    rows = {}

    def add(name, ms, amount, bound):
        if not ms or ms <= 0 or amount is None:
            return
        if bound == "alu":
            ach = amount / (ms * 1e-3) / 1e12
            row = {"bound": "alu", "ms": ms, "flops": amount, "achieved": ach, "peak": peak_alu, "unit": "TFLOP/s",
                   "frac": ach / peak_alu}
            if peaks:
                ap = peaks["fp64_fma_peak_tflops" if fp64 else "fp32_fma_peak_tflops"]
                row.update(achievable_peak=ap, frac_of_achievable=ach / ap)
        else:
            ach = amount / (ms * 1e-3) / 1e9
            row = {"bound": "hbm", "ms": ms, "bytes": amount, "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                   "frac": ach / PEAK_HBM_GBS}
            if peaks:
                row.update(achievable_peak=peaks["copy_gbs"], frac_of_achievable=ach / peaks["copy_gbs"])
        rows[name] = row

    evals = float(np.sum(st["evals"]))
    add("k_flatten", kernels.get("flatten_ms"), flat_bytes, "hbm")
    add("k_seed", kernels.get("seed_ms"), 16.0 * float(st["items"][0]) + 24.0 * n_pairs, "hbm")
    add("k_level", kernels.get("levels_ms"), flops_per_eval(n_iter) * evals, "alu")
    add("k_fine", kernels.get("fine_flatten_ms"), FLATTEN_BYTES_PER_TRI * float(st.get("fine_records", 0)), "hbm")
    if not kernels.get("certify_ms"):
        add("k_near", kernels.get("near_ms"), exact_pair_flops() * float(st["fallback"]), "alu")
    if kernels.get("backward_ms"):
        add("k_backward", kernels["backward_ms"], (32 + 10 * sz) * float(st["contacts"]) + 6 * sz * touched_verts,
            "hbm")
    weighted = sum(r["ms"] * r["frac"] for r in rows.values()) / ms_step
    return {"weighted_frac": weighted, "ms_step": ms_step, "ms_in_these_kernels": sum(r["ms"] for r in rows.values()),
            "kernels": rows}


def measure_peaks(torch, log=print) -> dict:
    """Achievable peaks of this GPU from the project's microbenchmarks
    (libpeak.so): FP32 and FP64 VALU loops over every SIMD (16 independent
    chains per lane, 8 waves per SIMD) -- FMA with uniform (SGPR) operands,
    FMA with three VGPR operands in the accumulating two-operand encoding
    (VOP2 FMAC) and in the three-operand encoding (VOP3), and FP32 add,
    multiply, max and three-input max -- and a 1 GiB device-to-device copy.  For each FP32 kind: the
    issue cycles of one wave64 instruction on a SIMD at the published
    2.4 GHz clock."""
    lib = C.CDLL(os.path.join(ROOT, "paper_2105_12415_amd", "libpeak.so"))
    lib.peak_fma.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_void_p]
    lib.peak_fma_per_lane.argtypes = [C.c_int]
    lib.peak_fma_per_lane.restype = C.c_longlong
    lib.peak_copy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int, C.c_void_p]
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    blocks = 256 * 8  # 256 CUs x 8 blocks of 4 waves = 8 waves per SIMD

    def timed(fn, reps):
        best = None
        for rep in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            rc = fn()
            e1.record()
            torch.cuda.synchronize()
            if rc:
                raise RuntimeError(f"microbenchmark launch failed ({rc})")
            ms = e0.elapsed_time(e1)
            if rep > 0 and (best is None or ms < best):
                best = ms
        return best

    out = {}
    # (name, fp64, kind, flop per operation, VALU instructions per operation:
    # a two-input max also canonicalises one input)
    kinds = (("fp32_fma_sgpr", 0, 0, 2, 1), ("fp32_fmac", 0, 1, 2, 1), ("fp32_add", 0, 2, 1, 1),
             ("fp32_mul", 0, 3, 1, 1), ("fp32_max", 0, 4, 1, 2), ("fp32_fma_vop3", 0, 5, 2, 1),
             ("fp32_max3", 0, 6, 2, 1), ("fp64_fma_sgpr", 1, 0, 2, 1), ("fp64_fmac", 1, 1, 2, 1))
    for name, fp64, kind, flop, ipo in kinds:
        iters = 10000 if fp64 else 20000
        buf = torch.empty(blocks * 256, dtype=torch.float64 if fp64 else torch.float32, device="cuda")
        ms = timed(lambda: lib.peak_fma(fp64, kind, blocks, iters, C.c_void_p(buf.data_ptr()), stream), 4)
        ops = blocks * 256 * lib.peak_fma_per_lane(iters)
        out[f"{name}_tflops"] = flop * ops / (ms * 1e-3) / 1e12
        out[f"{name}_cycles_per_wave64"] = ms * 1e-3 * 2.4e9 * 1024 / (blocks * 4 * ipo * lib.peak_fma_per_lane(iters))
    out["fp32_fma_peak_tflops"] = max(out["fp32_fma_sgpr_tflops"], out["fp32_fmac_tflops"],
                                      out["fp32_fma_vop3_tflops"])
    out["fp64_fma_peak_tflops"] = max(out["fp64_fma_sgpr_tflops"], out["fp64_fmac_tflops"])
    n = 1 << 30
    a = torch.empty(n, dtype=torch.uint8, device="cuda")
    b = torch.empty(n, dtype=torch.uint8, device="cuda")
    a.fill_(1)
    ms = timed(lambda: lib.peak_copy(C.c_void_p(a.data_ptr()), C.c_void_p(b.data_ptr()), n, 256 * 16, stream), 5)
    out["copy_gbs"] = 2.0 * n / (ms * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    log("[bench] peaks: " + ", ".join(f"{k} {v:.2f}" for k, v in out.items()))
    return out


def workload(name: str):
    import scenegen as sg
    if name not in WORKLOADS:
        raise SystemExit(f"unknown workload {name}; one of {sorted(WORKLOADS)}")
    make = {"two_spheres_s3_f64": sg.two_spheres_s3_f64, "two_spheres_s5": sg.two_spheres_s5_hier, "lattice": sg.lattice1000,
            "lattice_fwd_bwd": sg.lattice1000, "big_small": sg.big_plus_small,
            "lattice_frontier": sg.lattice1000, "lattice_forces": sg.lattice1000}[name]
    desc, backward = WORKLOADS[name]
    return make(), desc, backward


class Step:
    """One step: a seeded rigid perturbation of every particle (passed to the
    library as per-particle poses, applied while flattening), then the
    contact path (forward, and backward for the fwd+bwd workload)."""

    def __init__(self, ds, eng, backward: bool, n_steps: int, torch):
        import scenegen as sg
        self.ds, self.eng, self.backward = ds, eng, backward
        P = ds.n_particles
        centres = np.array([p.centre for p in ds.scene.particles])
        Rs, ts = sg.rigid_perturbations(P, max(n_steps, 1))
        # world = c + R (v - c) + t = R v + (c + t - R c)
        shift = centres + ts - np.einsum("kpij,pj->kpi", Rs, centres)
        poses = np.concatenate([Rs.reshape(len(Rs), P, 9), shift], axis=2)
        self.poses = torch.as_tensor(poses, device=ds.device, dtype=ds.dtype).contiguous()
        self.grad = torch.zeros(3, ds.n_verts, dtype=ds.dtype, device=ds.device)
        # a device status word per step, so that a flag raised by any step of
        # a replayed graph is seen (each call clears the word it writes)
        self.status_words = torch.zeros(len(self.poses), dtype=torch.int32, device=ds.device)

    def pose(self, k: int):
        self.ds.set_pose(self.poses[k % len(self.poses)])
        self.eng.status = self.status_words[k % len(self.poses):k % len(self.poses) + 1]

    def check_all(self, what: str):
        torch = sys.modules["torch"]
        torch.cuda.synchronize()
        w = self.status_words.cpu().numpy().astype(np.int64) & 0xFFFFFFFF
        bad = np.nonzero(w)[0]
        if len(bad):
            raise RuntimeError(f"device status {int(w[bad[0]]):#x} at step {int(bad[0])} {what}")

    def __call__(self, k: int):
        self.pose(k)
        self.eng.forward(with_energy=True)
        if self.backward:
            self.grad.zero_()
            self.eng.backward(self.grad)


class FrontierStep(Step):
    """One step on persistent active sets: the seeded rigid perturbation,
    dem_frontier_step (contacts of this step, widening / narrowing for the
    next) and the backward pass of its contacts."""

    def __call__(self, k: int):
        self.pose(k)
        self.eng.step(with_energy=True)
        if self.backward:
            self.grad.zero_()
            self.eng.backward(self.grad)


FRONTIER_SLOTS = ("reset", "flatten", "eval", "near", "group", "scan", "emit", "finish", "fold")


def frontier_kernel_times(torch, step: FrontierStep, K: int):
    """Per-launch durations (ms) of dem_frontier_step's kernels over K eager
    steps (HIP events recorded by the library between its launches), the
    backward call, and the step's counters averaged."""
    eng = step.eng
    n_ev = 16
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(n_ev)]
    for e in evs:
        e.record()
    torch.cuda.synchronize()
    handles = (C.c_void_p * n_ev)(*[C.c_void_p(e.cuda_event) for e in evs])
    eng.p.events = C.cast(handles, C.POINTER(C.c_void_p))
    eng.p.n_events = n_ev
    names = list(FRONTIER_SLOTS)
    if eng.p.certify:
        names.insert(3, "certify")
    acc = np.zeros(len(names))
    bwd = 0.0
    stats_acc = {}
    b0, b1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    try:
        for k in range(K):
            step.pose(k)
            eng.step(with_energy=True)
            step.grad.zero_()
            b0.record()
            eng.backward(step.grad)
            b1.record()
            torch.cuda.synchronize()
            status = eng.check()
            if status:
                raise RuntimeError(f"device status {status:#x} in eager frontier step {k}")
            for i in range(len(names)):
                acc[i] += evs[i].elapsed_time(evs[i + 1])
            bwd += b0.elapsed_time(b1)
            for k2, v in eng.stats_dict().items():
                v = np.array(v, dtype=np.float64) if isinstance(v, np.ndarray) else float(v)
                stats_acc[k2] = stats_acc.get(k2, 0) + v
    finally:
        eng.p.events = None
        eng.p.n_events = 0
    return dict(zip(names, acc / K)), bwd / K, {k2: v / K for k2, v in stats_acc.items()}


def time_graph(torch, step: Step, K: int, warmup: int):
    """Capture K steps in one graph; returns (ms/step by events, by wall clock)."""
    for w in range(warmup):
        step(w)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step(0)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for k in range(K):
            step(k)
    g.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record()
    g.replay()
    e1.record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / K
    return e0.elapsed_time(e1) / K, wall, g


def kernel_times(torch, step: Step, K: int):
    """Per-launch durations (ms) of dem_find_contacts' kernels, averaged over
    K eager steps, from HIP events the library records between launches on
    the step's stream; plus the backward call bracketed the same way."""
    from paper_2105_12415_amd import _abi
    eng = step.eng
    n_ev = 8 + 2 * _abi.DEM_MAX_LEVELS
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(n_ev)]
    for e in evs:
        e.record()  # materialise the underlying hipEvent
    torch.cuda.synchronize()
    handles = (C.c_void_p * n_ev)(*[C.c_void_p(e.cuda_event) for e in evs])
    eng.p.events = C.cast(handles, C.POINTER(C.c_void_p))
    eng.p.n_events = n_ev
    # slots: reset, flatten, seed, (descent, lazy flatten) per depth or the
    # flat kernel, certify (if on), fallback
    # (+1: the statistics fold after the exact pass)
    if eng.p.mode == _abi.DEM_MODE_HIER and eng.p.persistent:
        n_launch = 3 + (2 if eng.p.certify else 1) + 1  # reset, flatten, persistent descent, certify, fallback
    else:
        n_launch = 3 + (2 * eng.ds.n_levels_max if eng.p.mode == _abi.DEM_MODE_HIER else 1) + (2 if eng.p.certify else 1) + 1
    acc = np.zeros(n_launch)
    bwd = 0.0
    evals = np.zeros(_abi.DEM_MAX_LEVELS)
    stats_acc = None
    b0, b1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    try:
        for k in range(K):
            step.pose(k)
            eng.forward(with_energy=True)
            if step.backward:
                step.grad.zero_()
                b0.record()
                eng.backward(step.grad)
                b1.record()
            torch.cuda.synchronize()
            status = eng.check()
            if status:
                raise RuntimeError(f"device status {status:#x} in eager step {k}")
            for i in range(n_launch):
                acc[i] += evs[i].elapsed_time(evs[i + 1])
            if step.backward:
                bwd += b0.elapsed_time(b1)
            st = eng.stats_dict()
            if stats_acc is None:
                stats_acc = {k2: (np.array(v, dtype=np.float64) if isinstance(v, np.ndarray) else float(v))
                             for k2, v in st.items()}
            else:
                for k2, v in st.items():
                    stats_acc[k2] = stats_acc[k2] + (np.array(v, dtype=np.float64) if isinstance(v, np.ndarray) else v)
    finally:
        eng.p.events = None
        eng.p.n_events = 0
    for k2 in stats_acc:
        stats_acc[k2] = stats_acc[k2] / K
    return acc / K, bwd / K, stats_acc


from paper_2105_12415_amd.autotune import STORED as TUNE_CACHE  # noqa: E402


def run_mode(torch, api, ds, mode, backward, K, warmup, params_kw, contact_capacity, tune="cache",
             tune_out=None, half_depths=0):
    """tune: "cache" (parameters the autotuner stored for this scene, else
    time them now), "live" (time them now) or "off" (library defaults)."""
    from paper_2105_12415_amd import autotune
    p = api.make_params(mode, **params_kw)
    eng = api.ContactEngine(ds, p, contact_capacity=contact_capacity, energy_k=1e4)
    step = Step(ds, eng, backward, K, torch)
    # size the buffers on the first (eager) step: overflow triggers a regrow
    step.pose(0)
    eng.run()
    status = eng.check()
    if status:
        raise RuntimeError(f"device status {status:#x}")
    eng.tuned = None
    if tune != "off":
        space = None
        if mode == "flat":
            space = {"flat_tile_i": (256, 128), "omega": (1.0, 0.5)}
        space = {k: v for k, v in (space or autotune.hier_space(ds.n_levels_max)).items()
                 if k not in params_kw}
        cache = TUNE_CACHE if (tune == "cache" and mode == "hier" and not params_kw) else None
        best, log = autotune.tune_engine(eng, lambda: step(0), space=space, reps=1 if mode == "flat" else 7,
                                         cache=cache, write_cache=False)
        eng.tuned = {"chosen": best, "candidates": len(log),
                     "source": "stored by the autotuner" if (cache and not log) else "timed now"}
        if tune_out and log and mode == "hier":
            autotune.store(tune_out, autotune.signature(eng), best)
        step.pose(0)
        eng.run()
    if half_depths and mode == "hier":
        eng.p.half_depths = half_depths
        step.pose(0)
        eng.run()
    step.status_words.zero_()
    ms_graph, ms_wall, graph = time_graph(torch, step, K, warmup)
    step.check_all("after graph replay")
    kt, bwd_ms, st = kernel_times(torch, step, K)
    del graph
    return eng, step, ms_graph, ms_wall, kt, bwd_ms, st


def launch_knobs(eng) -> dict:
    """Every tunable launch/tile knob of the engine's parameters."""
    from paper_2105_12415_amd import autotune
    knobs = {k: autotune.get_knob(eng.p, k) for k in autotune.hier_space(eng.ds.n_levels_max)}
    if eng.p.half_depths:
        knobs["half_depths"] = eng.p.half_depths
    return knobs


def kernel_sources_sha256() -> str:
    h = hashlib.sha256()
    for f in ("dem_kernels.hip", "dem_geom.hpp"):
        h.update(open(os.path.join(ROOT, "paper_2105_12415_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def measured_traffic(workload: str, kernel: str, launch: dict, profiles_dir: str = None):
    """HBM bytes per launch of ``kernel`` from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary of this workload (already scaled by the
    copy calibration), if it was taken on these kernel sources with these
    launch parameters; else (None, reason)."""
    path = os.path.join(profiles_dir or os.path.join(ROOT, "profiles"), f"hbm_traffic_{workload}.md")
    if not os.path.exists(path):
        return None, "no counter summary for this workload"
    rec = None
    for line in open(path):
        if line.startswith("traffic-json: "):
            rec = json.loads(line[len("traffic-json: "):])
    if rec is None or kernel not in rec.get("per_dispatch", {}):
        return None, "counter summary lacks this kernel"
    if rec.get("source_sha256") != kernel_sources_sha256():
        return None, "kernel sources changed since the counters were taken"
    prof = rec.get("launch", {})
    if any(abs(float(prof.get(k, -1)) - float(v)) > 1e-6 for k, v in launch.items()):
        return None, "launch parameters differ from the profiled run"
    d = rec["per_dispatch"][kernel]
    return d["read_bytes"] + d["write_bytes"], "rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated"


def frontier_launch(p) -> dict:
    return {k: getattr(p, k) for k in ("grid", "frontier_grid", "block", "omega", "n_iter", "certify", "prune_exact")}


def run_frontier_bench(torch, api, ds, args, params_kw, desc, log):
    """lattice_frontier: persistent active sets followed through K perturbed
    steps (captured in one HIP graph) after converging at the start pose."""
    from paper_2105_12415_amd import autotune
    K = args.steps
    p = api.make_params("hier", **params_kw)
    eng = api.FrontierEngine(ds, p, contact_capacity=args.contact_capacity, energy_k=1e4)
    tuned = None
    if not args.no_autotune and not params_kw:
        # the descent's stored launch shape and damping for this scene
        rec = autotune.apply_stored(eng)
        tuned = {"chosen": rec, "source": "stored by the autotuner (descent)"} if rec else None
    step = FrontierStep(ds, eng, True, K, torch)
    step.pose(0)
    eng.init()
    t0 = time.perf_counter()
    n_conv = eng.run_to_fixed_point()
    st0 = eng.stats_dict()
    n_leaves = int(eng.state_host()[1])
    log(f"[bench] frontier converged in {n_conv} steps ({time.perf_counter() - t0:.1f} s): {n_leaves} leaves, "
        f"{eng.count()} contacts")
    # room for the sets, the near list and the contacts to follow the motion inside the graph
    eng.reserve(int(1.5 * n_leaves) + 4096)
    eng.p.near_capacity = max(int(eng.p.near_capacity), 8 * int(st0["near"]) // 2 + 8 * 65536)
    eng.ws = None
    eng._alloc_ws()
    if eng.contacts.capacity < 2 * eng.count():
        eng.contacts = api.ContactBuffers.alloc(2 * eng.count(), ds.dtype, ds.device)
    for k in range(K):
        step(k)
        status = eng.check()
        if status:
            raise RuntimeError(f"device status {status:#x} in eager frontier step {k}")
    step.status_words.zero_()
    ms, ms_wall, graph = time_graph(torch, step, K, args.warmup)
    step.check_all("after graph replay")
    del graph
    kt, bwd_ms, st = frontier_kernel_times(torch, step, K)
    evals = float(st["frontier_leaves"])
    log(f"[bench] frontier: {ms:.3f} ms/step (wall {ms_wall:.3f}), {evals:.4g} leaves/step, "
        f"{st['contacts']:.0f} contacts, unfolded {st['frontier_unfolded']:.1f}, "
        f"collapsed {st['frontier_collapsed']:.1f}")
    n_iter = eng.p.n_iter
    flops = flops_per_eval(n_iter) * evals
    achieved = flops / (kt["eval"] * 1e-3) / 1e12
    launch = frontier_launch(eng.p)
    traffic, traffic_note = measured_traffic(args.workload, "k_fr_eval", launch)
    roof = {"bound": "alu", "kernel": "k_fr_eval<float>", "achieved": achieved, "peak": PEAK_FP32_VALU_TFLOPS,
            "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_VALU_TFLOPS, "traffic": traffic,
            "traffic_note": traffic_note, "launches_per_step": 1, "avg_launch_ms": kt["eval"],
            "flops_per_eval": flops_per_eval(n_iter), "evals_per_step": evals}
    L = ds.n_levels_max
    out = {"metric": METRIC, "value": evals / (ms * 1e-3), "unit": "tri-pair evals/s", "n_gpus": 1,
           "steps": K, "warmup": args.warmup, "ms_per_step": ms, "ms_per_step_wall": ms_wall,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": f"{args.workload}: {desc}; forward + backward (k=1e4), per-step rigid "
                      f"perturbation, {K} steps captured in one HIP graph after converging the active sets "
                      f"at the start pose ({n_conv} steps)",
                      "particles": ds.n_particles, "triangles_all_levels": ds.n_tris,
                      "candidate_pairs": ds.n_pairs, "fine_pairs": ds.n_fine_pairs(), "n_iter": n_iter,
                      "autotuned": tuned, "launch": launch},
           "roofline": roof,
           "kernels": dict({f"{k}_ms": v for k, v in kt.items()}, backward_ms=bwd_ms),
           "stats": {"leaves": evals, "leaves_by_depth": [int(x) for x in st["evals"][:L]],
                     "unfolded": st["frontier_unfolded"], "collapsed": st["frontier_collapsed"],
                     "near": st["near"], "contacts": st["contacts"],
                     "converged_leaves": n_leaves, "converge_steps": n_conv}}
    del eng, step
    torch.cuda.empty_cache()
    if not args.no_flat:
        # the full descent on the same perturbed steps, for comparison
        de, dstep, dms, dwall, dkt, dbwd, dst = run_mode(torch, api, ds, "hier", True, K, args.warmup, params_kw,
                                                       args.contact_capacity,
                                                       tune="off" if args.no_autotune else "cache")
        out["descent"] = {"ms_per_step": dms, "evals_per_step": float(np.sum(dst["evals"])),
                          "contacts": dst["contacts"]}
        out["speedup_vs_descent"] = dms / ms
        log(f"[bench] descent: {dms:.3f} ms/step")
        del de, dstep
    return out


FORCE_BYTES_PER_CONTACT = 48  # pi, pj, ti, tj, x, n of a contact (40 B) + its two epsilons (8 B)
FORCE_BYTES_PER_MERGED = 56   # pi, pj, members, x, n, f of a merged contact (FP32)


def run_forces_bench(torch, api, ds, scene, args, params_kw, desc, log):
    """lattice_forces: contacts (dem_find_contacts) then dem_contact_forces
    (merging, force law, per-particle force and torque) per perturbed step."""
    from paper_2105_12415_amd import autotune
    K = args.steps
    p = api.make_params("hier", **params_kw)
    eng = api.ContactEngine(ds, p, contact_capacity=args.contact_capacity, energy_k=1e4)
    if not args.no_autotune and not params_kw:
        autotune.apply_stored(eng)
    step = Step(ds, eng, False, K, torch)
    step.pose(0)
    eng.run()
    mass = torch.as_tensor(np.array([q.radius ** 3 for q in scene.particles]), dtype=ds.dtype, device=ds.device)
    centre = torch.as_tensor(np.array([q.centre for q in scene.particles]).T.copy(), dtype=ds.dtype,
                             device=ds.device)
    fe = api.ForceEngine(ds, eng.contacts.capacity)

    def fstep(k):
        step(k)
        fe.run(eng.contacts, mass, centre, with_group=False)

    for k in range(K):
        fstep(k)
        if eng.check() or fe.check():
            raise RuntimeError(f"device status {eng.check():#x} / {fe.check():#x} in eager step {k}")
    step.status_words.zero_()
    ms_fwd, _, g0 = time_graph(torch, step, K, args.warmup)
    step.check_all("after graph replay (contacts)")
    del g0
    ms, ms_wall, g1 = time_graph(torch, fstep, K, args.warmup)
    step.check_all("after graph replay (contacts + forces)")
    del g1
    if fe.check():
        raise RuntimeError(f"device status {fe.check():#x} after graph replay")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    f_ms, n_c, n_m = 0.0, 0, 0
    for k in range(K):
        step(k)
        e0.record()
        fe.run(eng.contacts, mass, centre, with_group=False)
        e1.record()
        torch.cuda.synchronize()
        f_ms += e0.elapsed_time(e1)
        n_c += eng.count()
        n_m += int(fe.merged.count.item())
    f_ms, n_c, n_m = f_ms / K, n_c / K, n_m / K
    st = eng.stats_dict()
    evals = float(np.sum(st["evals"]))
    log(f"[bench] forces: step {ms:.3f} ms (contacts only {ms_fwd:.3f}); force pass {f_ms:.3f} ms for "
        f"{n_c:.0f} contacts -> {n_m:.0f} merged")
    bytes_ = FORCE_BYTES_PER_CONTACT * n_c + FORCE_BYTES_PER_MERGED * n_m
    achieved = bytes_ / (f_ms * 1e-3) / 1e9
    return {"metric": METRIC, "value": evals / (ms * 1e-3), "unit": "tri-pair evals/s", "n_gpus": 1, "steps": K,
            "warmup": args.warmup, "ms_per_step": ms, "ms_per_step_wall": ms_wall, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"{args.workload}: {desc}; per-step rigid perturbation, {K} steps captured in "
                       "one HIP graph (contacts + forces)", "particles": ds.n_particles,
                       "triangles_all_levels": ds.n_tris, "candidate_pairs": ds.n_pairs, "k_s": 1000.0,
                       "merge_scale": 1.0, "mass": "radius^3", "centre": "particle centre"},
            "roofline": {"bound": "hbm", "kernel": "dem_contact_forces (all kernels of the pass)",
                         "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS,
                         "traffic": None, "traffic_note": "no counter summary for this pass",
                         "bytes_per_contact": FORCE_BYTES_PER_CONTACT, "bytes_per_merged": FORCE_BYTES_PER_MERGED},
            "forces": {"ms": f_ms, "contacts": n_c, "merged": n_m, "contacts_per_s": n_c / (f_ms * 1e-3),
                       "contacts_only_ms_per_step": ms_fwd}}


def forces_cpu_baseline(scene, n_sample: int):
    import oracle
    from oracle import forces as of
    fs = oracle.fine_scene(scene)
    rng = np.random.default_rng(12345)
    P = np.asarray(scene.pairs)
    idx = np.sort(rng.choice(len(P), min(n_sample, len(P)), replace=False))
    c = oracle.find_contacts(fs, pairs=P[idx])
    mass = np.array([q.radius ** 3 for q in scene.particles])
    centre = np.array([q.centre for q in scene.particles])
    t0 = time.perf_counter()
    r = of.contact_forces(fs, c, mass, centre, pairs=P[idx])
    dt = time.perf_counter() - t0
    return {"value": len(c["d"]) / dt, "unit": "contacts/s", "cores": 1, "kind": "oracle",
            "sample": f"force pass (merging, force law, per-particle sums) over the {len(c['d'])} contacts of "
                      f"{len(idx)} seeded candidate pairs ({len(r['f'])} merged) in {dt:.2f} s, FP64 numpy/scipy",
            "seconds": dt}


def cpu_baseline(scene, n_sample: int, backward: bool, n_single: int = 12):
    """The FP64 oracle on a seeded sample of candidate pairs: all host
    threads, then one thread on a seeded subset of that sample.  ``value``
    counts the triangle pairs the oracle actually evaluated exactly
    (``tested``: the pairs its exact bounding-sphere test did not reject),
    the same kind of unit as the GPU's evaluations; the fine pairs the sample
    covers (decided, most by the rejection test) are reported beside it."""
    import oracle
    fs = oracle.fine_scene(scene)
    rng = np.random.default_rng(12345)
    n = min(n_sample, len(scene.pairs))
    idx = np.sort(rng.choice(len(scene.pairs), n, replace=False))
    P = np.asarray(scene.pairs)[idx]
    F = fs.tri_count.astype(np.int64)

    def run(pairs, threads):
        t0 = time.perf_counter()
        c = oracle.find_contacts(fs, pairs=pairs, n_threads=threads)
        if backward:
            oracle.energy_grad(fs, c, 1e4, pairs=pairs)
        return c, time.perf_counter() - t0

    threads = oracle.default_threads()
    c, dt = run(P, threads)
    fine = int(np.sum(F[P[:, 0]] * F[P[:, 1]]))
    sub = P[np.sort(rng.choice(n, min(n_single, n), replace=False))]
    c1, dt1 = run(sub, 1)
    fine1 = int(np.sum(F[sub[:, 0]] * F[sub[:, 1]]))
    what = "exact FP64 triangle-pair distances" + (", plus energy gradient" if backward else "")
    return {"value": c["tested"] / dt, "unit": "tri-pair evals/s", "cores": threads, "kind": "oracle",
            "sample": (f"{n} of {len(scene.pairs)} candidate particle pairs (seeded): {fine} fine triangle "
                       f"pairs decided, {c['tested']} of them evaluated exactly ({what}; the rest rejected by "
                       f"the exact bounding-sphere test) in {dt:.2f} s on {threads} threads"),
            "seconds": dt, "tested": int(c["tested"]), "fine_pairs": fine, "fine_pairs_per_s": fine / dt,
            "contacts": int(len(c["d"])),
            "single_thread": {"value": c1["tested"] / dt1, "unit": "tri-pair evals/s", "cores": 1,
                              "sample": f"{len(sub)} of those pairs (seeded): {fine1} fine pairs, "
                                        f"{c1['tested']} evaluated exactly, in {dt1:.2f} s",
                              "seconds": dt1, "tested": int(c1["tested"]), "fine_pairs_per_s": fine1 / dt1}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="lattice_fwd_bwd", choices=sorted(WORKLOADS))
    ap.add_argument("--flat-steps", type=int, default=1)
    ap.add_argument("--no-flat", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-pairs", type=int, default=180)
    ap.add_argument("--contact-capacity", type=int, default=1 << 23)
    ap.add_argument("--param", action="append", default=[], help="dem_params override, e.g. omega=0.5")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default launch parameters")
    ap.add_argument("--retune", action="store_true",
                    help="time the autotuner's candidates now instead of using the stored result")
    ap.add_argument("--tune-out", default=None, help="write a result timed now to this JSON file")
    ap.add_argument("--half-depths", type=int, default=0,
                    help="run the descent's Newton iteration in half precision at tree depths below this "
                         "(applied on top of the stored launch parameters)")
    ap.add_argument("--peaks-only", action="store_true",
                    help="only run the achievable-peak microbenchmarks and print them as JSON")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="only run a plain device-to-device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.calib_copy_mib:
        import torch
        n = args.calib_copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calib_copy_bytes": 4 * n, "copies": 3}))
        return
    if args.peaks_only:
        import torch
        print(json.dumps(measure_peaks(torch)))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    from paper_2105_12415_amd import api

    params_kw = {}
    for kv in args.param:
        k, v = kv.split("=")
        params_kw[k] = float(v) if "." in v or "e" in v else int(v)

    scene, desc, backward = workload(args.workload)
    ds = api.DeviceScene(scene, device="cuda:0")
    K = args.steps
    log = lambda m: print(m, file=sys.stderr, flush=True)
    log(f"[bench] {args.workload}: {desc}; {ds.n_particles} particles, {ds.n_tris} triangles, "
        f"{ds.n_pairs} candidate pairs, {ds.n_fine_pairs()} fine pairs")

    if args.workload == "lattice_forces":
        out = run_forces_bench(torch, api, ds, scene, args, params_kw, desc, log)
        if not args.no_cpu:
            log("[bench] cpu baseline (oracle force pass) ...")
            out["cpu_baseline"] = forces_cpu_baseline(scene, args.cpu_pairs)
        print(json.dumps(out), flush=True)
        return
    if args.workload == "lattice_frontier":
        out = run_frontier_bench(torch, api, ds, args, params_kw, desc, log)
        if not args.no_cpu:
            log("[bench] cpu baseline (oracle) ...")
            out["cpu_baseline"] = cpu_baseline(scene, args.cpu_pairs, backward)
        print(json.dumps(out), flush=True)
        return

    eng, step, ms, ms_wall, kt, bwd_ms, st = run_mode(torch, api, ds, "hier", backward, K, args.warmup,
                                                     params_kw, args.contact_capacity,
                                                     tune="off" if args.no_autotune else
                                                     ("live" if args.retune else "cache"),
                                                     tune_out=args.tune_out, half_depths=args.half_depths)
    evals = float(np.sum(st["evals"]))
    log(f"[bench] hier: {ms:.3f} ms/step (wall {ms_wall:.3f}), {evals:.4g} evals/step, "
        f"{st['contacts']:.0f} contacts, near {st['near']:.0f}")
    L = ds.n_levels_max
    persistent = bool(eng.p.persistent)
    if persistent:
        # one launch: seeding, every depth and the lazy flattening
        level_kt, fine_kt, nb, seed_ms = kt[2:3], [], 3, None
    else:
        level_kt = kt[3:3 + 2 * L:2]   # descent launches
        fine_kt = kt[4:4 + 2 * L:2]    # lazy flattening after each depth
        nb, seed_ms = 3 + 2 * L, kt[2]
    level_ms = float(np.sum(level_kt))
    n_iter = eng.p.n_iter
    fl = flops_per_eval(n_iter) * evals
    dtype = "f64" if scene.dtype == "f64" else "f32"
    peak = PEAK_FP64_VALU_TFLOPS if dtype == "f64" else PEAK_FP32_VALU_TFLOPS
    achieved = fl / (level_ms * 1e-3) / 1e12
    launch = launch_knobs(eng)
    kname = "k_descent" if persistent else "k_level"
    traffic, traffic_note = measured_traffic(args.workload, kname, launch)
    roof = {"bound": "alu", "kernel": f"{kname}<{'double' if dtype == 'f64' else 'float'}>",
            "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
            "traffic": traffic, "traffic_note": traffic_note,
            "launches_per_step": len(level_kt), "avg_launch_ms": level_ms / len(level_kt),
            "flops_per_eval": flops_per_eval(n_iter), "evals_per_step": evals,
            "peak_published_packed_fp32": 157.3}
    n_written = ds.n_eager_records
    flat_bytes = (FLATTEN_BYTES_PER_TRI * n_written + FLATTEN_BYTES_SKIPPED * (ds.n_tris - n_written)
                  + FLATTEN_BYTES_PER_VERT * ds.n_verts)
    cert = bool(eng.p.certify)
    kernels = {"reset_ms": kt[0], "flatten_ms": kt[1], "fine_flatten_ms": float(np.sum(fine_kt)),
               "seed_ms": seed_ms, "levels_ms": level_ms,
               "levels_ms_each": [round(x, 4) for x in level_kt],
               "certify_ms": kt[nb] if cert else None, "fallback_ms": kt[nb + (1 if cert else 0)],
               "near_ms": float(np.sum(kt[nb:nb + (2 if cert else 1)])), "fold_ms": kt[-1],
               "backward_ms": bwd_ms if backward else None,
               "flatten_records": n_written, "flatten_GBs": flat_bytes / (kt[1] * 1e-3) / 1e9}
    out = {"metric": METRIC, "value": evals / (ms * 1e-3), "unit": "tri-pair evals/s", "n_gpus": 1,
           "steps": K, "warmup": args.warmup, "ms_per_step": ms, "ms_per_step_wall": ms_wall,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
           "data": "synthetic",
           "config": {"workload": f"{args.workload}: {desc}" + ("; forward + backward (k=1e4), "
                      f"per-step rigid perturbation, {K} steps captured in one HIP graph" if backward else
                      f"; forward contacts, {K} steps captured in one HIP graph"),
                      "particles": ds.n_particles, "triangles_all_levels": ds.n_tris,
                      "candidate_pairs": ds.n_pairs, "fine_pairs": ds.n_fine_pairs(), "n_iter": n_iter,
                      "autotuned": eng.tuned, "launch": launch},
           "roofline": roof, "kernels": kernels,
           "stats": {"evals_per_level": [int(x) for x in st["evals"][:L]],
                     "survivors_per_level": [int(x) for x in st["survivors"][:L]],
                     "near": st["near"], "certified": st["certified"], "fallback": st["fallback"],
                     "contacts": st["contacts"], "fine_records": st.get("fine_records", 0)}}
    # distinct vertices the backward's gradient touches (last eager step's contacts)
    touched = 0
    if backward:
        nc = eng.count()
        tvd = ds.tri_verts
        ti, tj = eng.contacts.ti[:nc].long(), eng.contacts.tj[:nc].long()
        touched = int(torch.unique(torch.cat([tvd[:, ti].reshape(-1), tvd[:, tj].reshape(-1)])).numel())
        out["stats"]["backward_vertices"] = touched
    if not args.no_flat:
        del eng, step
        torch.cuda.empty_cache()
        fe, fstep, fms, fwall, fkt, fbwd, fst = run_mode(torch, api, ds, "flat", backward, args.flat_steps,
                                                       0, params_kw, args.contact_capacity,
                                                       tune="off" if args.no_autotune else "live")
        fevals = float(np.sum(fst["evals"]))
        out["flat"] = {"autotuned": fe.tuned, "ms_per_step": fms, "ms_per_step_wall": fwall, "evals_per_step": fevals,
                       "evals_per_s": fevals / (fms * 1e-3), "contacts": fst["contacts"],
                       "flat_kernel_ms": float(fkt[3]), "near_ms": float(np.sum(fkt[4:-1])),
                       "flat_kernel_TFLOPs": flops_per_eval(n_iter) * fevals / (fkt[3] * 1e-3) / 1e12}
        out["speedup_vs_flat"] = fms / ms
        log(f"[bench] flat: {fms:.2f} ms/step, {fevals:.4g} evals/step")
        del fe, fstep
    # achievable peaks of this GPU (after the timed work), then every kernel
    # of the step against its roof
    peaks = measure_peaks(torch, log)
    out["peaks"] = peaks
    ap = peaks["fp64_fma_peak_tflops" if dtype == "f64" else "fp32_fma_peak_tflops"]
    roof["achievable_peak"] = ap
    roof["frac_of_achievable"] = achieved / ap
    roof["step"] = step_roofline(ms, kernels, st, ds.n_pairs, n_iter, dtype == "f64", flat_bytes, touched, peaks)
    log(f"[bench] step roofline: time-weighted fraction {roof['step']['weighted_frac']:.3f}")
    if not args.no_cpu:
        log("[bench] cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(scene, args.cpu_pairs, backward)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
