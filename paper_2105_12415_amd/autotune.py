"""Autotuner for the launch shape and tiling of the contact path.

Coordinate descent over a small space of dem_params knobs: each knob in
turn takes every candidate value while the others hold their best values so
far, and the fastest value stays.  Candidates are timed on the caller's own
scene and step (HIP events on the current stream, median of a few repeats
after a warm-up), so the choice reflects that workload's tree depths, item
shapes and contact density.

None of the knobs changes the result beyond the parity tolerances:
``block``, ``grid``, ``batch_items``, ``seed_chunk``, the per-depth
``level_grid.d`` / ``level_batch.d`` and the flat tiles only change how work
is laid out; ``omega`` damps the Newton step (the search direction of the
lower bound, hence only how much is pruned) and ``certify`` chooses between
two exact ways of settling near pairs.

A knob named ``array.index`` addresses one element of an array field of
dem_params (the per-depth launch shapes).
"""
from __future__ import annotations

import json
import os
from typing import Callable, Dict, List, Optional, Sequence, Tuple

HIER_SPACE: Dict[str, Sequence] = {
    "batch_items": (128, 64, 32),
    "grid": (1024, 2048, 4096),
    "block": (256, 128),
    "seed_chunk": (16, 8),
    "omega": (1.0, 0.7, 0.5),
    "certify": (0, 1),
}

LEVEL_GRIDS = (512, 1024, 1536, 2048, 3072)
LEVEL_BATCHES = (8, 16, 32, 64, 128, 256)


def hier_space(n_levels: int) -> Dict[str, Sequence]:
    """HIER_SPACE, then a grid and a batch size for each tree depth."""
    space = dict(HIER_SPACE)
    for d in range(n_levels):
        space[f"level_grid.{d}"] = LEVEL_GRIDS
        space[f"level_batch.{d}"] = LEVEL_BATCHES
    return space


def get_knob(p, name: str):
    if "." in name:
        field, idx = name.split(".")
        return getattr(p, field)[int(idx)]
    return getattr(p, name)


def set_knob(p, name: str, value) -> None:
    if "." in name:
        field, idx = name.split(".")
        getattr(p, field)[int(idx)] = value
    else:
        setattr(p, name, value)


FLAT_SPACE: Dict[str, Sequence] = {
    "flat_tile_i": (256, 128),
    "grid": (2048, 1024, 4096),
    "omega": (1.0, 0.5),
}


def coordinate_descent(measure: Callable[[Dict], float], start: Dict, space: Dict[str, Sequence],
                       sweeps: int = 1) -> Tuple[Dict, List[Tuple[Dict, float]]]:
    """Minimise measure(params) one knob at a time; returns (best, log)."""
    best = dict(start)
    best_t = measure(best)
    log = [(dict(best), best_t)]
    seen = {tuple(sorted(best.items()))}
    for _ in range(sweeps):
        for knob, values in space.items():
            for v in values:
                cand = dict(best)
                cand[knob] = v
                key = tuple(sorted(cand.items()))
                if key in seen:
                    continue
                seen.add(key)
                t = measure(cand)
                log.append((dict(cand), t))
                if t < best_t:
                    best, best_t = cand, t
    return best, log


def time_step(step: Callable[[], None], reps: int = 5, warmup: int = 1) -> float:
    """Median milliseconds of step() on the current stream (HIP events)."""
    import torch
    for _ in range(warmup):
        step()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        step()
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    ts.sort()
    return ts[len(ts) // 2]


STORED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_params.json")


def apply_stored(engine, path: str = STORED) -> Optional[Dict]:
    """Apply the stored tuning result for the engine's scene (the launch
    parameters the benchmark times), if there is one; returns it."""
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path)).get(signature(engine))
    except (OSError, ValueError):
        return None
    if rec:
        for k, v in rec.items():
            set_knob(engine.p, k, v)
    return rec


def signature(engine) -> str:
    """Key of a tuning result: scene sizes, precision, mode and N_it."""
    ds, p = engine.ds, engine.p
    return f"{ds.n_tris}:{ds.n_verts}:{ds.n_pairs}:{ds.precision}:{p.mode}:{p.n_iter}"


def store(path: str, sig: str, best: Dict) -> None:
    """Add (or replace) one tuning result in the JSON file at path."""
    data = {}
    if os.path.exists(path):
        try:
            data = json.load(open(path))
        except (OSError, ValueError):
            data = {}
    data[sig] = {k: (float(v) if isinstance(v, float) else int(v)) for k, v in best.items()}
    with open(path, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)


def tune_engine(engine, step: Callable[[], None], space: Optional[Dict[str, Sequence]] = None,
                reps: int = 5, cache: Optional[str] = None,
                write_cache: bool = True) -> Tuple[Dict, List[Tuple[Dict, float]]]:
    """Tune engine.p in place for ``step`` (which must call engine.forward()).

    The chosen values are applied to engine.p and returned; ``cache`` (a
    JSON path) holds results keyed by a signature of the scene and mode: a
    stored result is applied without timing (the returned log is then
    empty), otherwise the timed result is added to it (if write_cache).
    """
    from . import _abi
    p = engine.p
    ds = engine.ds
    if space is None:
        space = hier_space(ds.n_levels_max) if p.mode == _abi.DEM_MODE_HIER else FLAT_SPACE
    sig = signature(engine)
    if cache and os.path.exists(cache):
        try:
            stored = json.load(open(cache)).get(sig)
        except (OSError, ValueError):
            stored = None
        if stored:
            for k, v in stored.items():
                set_knob(p, k, v)
            return stored, []
    start = {k: get_knob(p, k) for k in space}

    def measure(cand: Dict) -> float:
        for k, v in cand.items():
            set_knob(p, k, v)
        try:
            t = time_step(step, reps=reps)
        except _abi.DemError:
            return float("inf")  # an invalid combination (e.g. batch > block)
        status = engine.check()
        if status:
            return float("inf")  # e.g. a capacity overflow: never prefer it
        return t

    # two sweeps: a knob chosen early (the global grid) is revisited once the
    # per-depth knobs have taken over the launches it first decided
    best, log = coordinate_descent(measure, start, space, sweeps=2)
    for k, v in best.items():
        set_knob(p, k, v)
    if cache and write_cache:
        store(cache, sig, best)
    return best, log
