"""The autotuner's search (CPU) and its effect on results (GPU)."""
import numpy as np
import pytest

from paper_2105_12415_amd import autotune


def test_coordinate_descent_finds_separable_minimum():
    space = {"a": (1, 2, 3), "b": (10, 20), "c": (0.5, 1.0)}
    cost = lambda p: (p["a"] - 2) ** 2 + (p["b"] - 20) ** 2 / 100 + abs(p["c"] - 0.5)
    best, log = autotune.coordinate_descent(cost, {"a": 1, "b": 10, "c": 1.0}, space)
    assert best == {"a": 2, "b": 20, "c": 0.5}
    assert len(log) == 1 + 2 + 1 + 1  # start + the other values of each knob


def test_coordinate_descent_never_prefers_failures():
    space = {"a": (1, 2, 3)}
    cost = lambda p: float("inf") if p["a"] == 3 else float(p["a"])
    best, _ = autotune.coordinate_descent(cost, {"a": 2}, space)
    assert best == {"a": 1}


def test_per_depth_knobs_address_param_arrays():
    from paper_2105_12415_amd import _abi
    p = _abi.default_params()
    space = autotune.hier_space(3)
    assert "level_grid.2" in space and "level_batch.0" in space and "level_grid.3" not in space
    autotune.set_knob(p, "level_grid.2", 1536)
    autotune.set_knob(p, "level_batch.0", 64)
    autotune.set_knob(p, "grid", 2048)
    assert p.level_grid[2] == 1536 and p.level_batch[0] == 64 and p.grid == 2048
    assert autotune.get_knob(p, "level_grid.2") == 1536 and autotune.get_knob(p, "level_grid.1") == 0


@pytest.mark.gpu
def test_tuned_parameters_keep_the_contacts():
    import scenegen as sg
    from paper_2105_12415_amd import api
    scene = sg.two_spheres(4, [1, 2, 3, 4], "f32", sep=2.03, stream_id=51, name="tune")
    ds = api.DeviceScene(scene, device="cuda:0")
    ref = api.ContactEngine(ds, api.make_params("hier"))
    assert ref.run() == 0
    r0 = ref.result()
    eng = api.ContactEngine(ds, api.make_params("hier"))
    assert eng.run() == 0
    best, log = autotune.tune_engine(eng, lambda: eng.forward(), reps=2)
    assert len(log) > 5 and set(best) == set(autotune.hier_space(ds.n_levels_max))
    assert eng.run() == 0
    r1 = eng.result()
    k0 = set(zip(r0["ti"].tolist(), r0["tj"].tolist()))
    k1 = set(zip(r1["ti"].tolist(), r1["tj"].tolist()))
    assert k0 == k1
    assert abs(r1["energy"] - r0["energy"]) <= 1e-5 * r0["energy"]
