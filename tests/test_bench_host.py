"""Host logic of bench.py: the roofline traffic is taken from a committed
counter summary only while it matches the kernel sources and the launch
parameters it was measured with."""
import json

import bench


def _write(tmp_path, sha, launch):
    rec = {"source_sha256": sha, "workload": "w", "launch": launch,
           "per_dispatch": {"k_level": {"read_bytes": 1000.0, "write_bytes": 24.0}}}
    (tmp_path / "hbm_traffic_w.md").write_text("# summary\n\ntraffic-json: " + json.dumps(rec) + "\n")


def test_traffic_only_for_matching_sources_and_launch(tmp_path):
    launch = {"grid": 1024, "omega": 0.5}
    _write(tmp_path, bench.kernel_sources_sha256(), launch)
    t, note = bench.measured_traffic("w", "k_level", launch, str(tmp_path))
    assert t == 1024.0, note
    t, note = bench.measured_traffic("w", "k_level", {"grid": 2048, "omega": 0.5}, str(tmp_path))
    assert t is None and "launch" in note
    _write(tmp_path, "0" * 64, launch)
    t, note = bench.measured_traffic("w", "k_level", launch, str(tmp_path))
    assert t is None and "sources" in note
    t, note = bench.measured_traffic("absent", "k_level", launch, str(tmp_path))
    assert t is None


def test_flops_per_eval_counts():
    # 74 per Newton iteration, 24 saved by the first, 84 for set-up, clamp and bound
    assert bench.flops_per_eval(4) == 356
    assert bench.flops_per_eval(0) == 84
    assert bench.flops_per_eval(1) == 134


def test_exact_pair_flops_count():
    # set-up 94, crossings 314, vertex-interior 178, edge lengths 42, nine
    # segment pairs 765, winner 35, emission 24
    assert bench.exact_pair_flops() == 1452


def test_step_roofline_weights_each_kernel_by_time():
    """Two kernels of a 2 ms step: a descent at half the FP32 VALU peak for
    1 ms and a backward at a quarter of HBM for 0.5 ms give 0.3125."""
    import numpy as np
    peak = bench.PEAK_FP32_VALU_TFLOPS
    evals = 0.5 * peak * 1e12 * 1e-3 / bench.flops_per_eval(4)
    contacts = 1000.0
    per_contact = 32 + 10 * 4
    bwd_bytes = 0.25 * bench.PEAK_HBM_GBS * 1e9 * 0.5e-3
    touched = (bwd_bytes - per_contact * contacts) / 24
    st = {"evals": np.array([evals]), "items": np.array([0.0]), "fallback": 0.0, "contacts": contacts,
          "fine_records": 0}
    r = bench.step_roofline(2.0, {"levels_ms": 1.0, "backward_ms": 0.5}, st, 0, 4, False, 0.0, touched)
    assert abs(r["kernels"]["k_level"]["frac"] - 0.5) < 1e-9
    assert abs(r["kernels"]["k_backward"]["frac"] - 0.25) < 1e-9
    assert abs(r["weighted_frac"] - (1.0 * 0.5 + 0.5 * 0.25) / 2.0) < 1e-9


def _counter_csv(path, rows):
    """A rocprofv3 counter_collection.csv with (dispatch, kernel, counter, value) rows."""
    path.mkdir(parents=True, exist_ok=True)
    lines = ["Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value"]
    lines += [f'{d},"{k}",{c},{v}' for d, k, c, v in rows]
    (path / "p_counter_collection.csv").write_text("\n".join(lines) + "\n")


def test_traffic_summary_averages_a_kernel_family(tmp_path):
    """Two instantiations of one kernel (one launch per depth, the deepest
    depth in its own variant) give one per-dispatch figure: the family's
    bytes over all of its dispatches, each scaled by the copy calibration."""
    from paper_2105_12415_amd import profile_summary as ps
    a = "void k_level<float, 4, 256, false, false>(SoupRec<float> const*, LevelArgs)"
    b = "void k_level<float, 4, 256, false, true>(SoupRec<float> const*, LevelArgs)"
    # five dispatches of a reading 10 KiB each, one of b reading 70 KiB; writes 1 and 7 KiB
    _counter_csv(tmp_path / "fetch", [(i, a, "FETCH_SIZE", 10.0) for i in range(5)] + [(5, b, "FETCH_SIZE", 70.0)])
    _counter_csv(tmp_path / "write", [(i, a, "WRITE_SIZE", 1.0) for i in range(5)] + [(5, b, "WRITE_SIZE", 7.0)])
    # calibration: a 1 MiB copy reads 512 KiB by the counter (scale 2) and writes 1024 KiB (scale 1)
    _counter_csv(tmp_path / "cf", [(0, "k_copy", "FETCH_SIZE", 512.0)])
    _counter_csv(tmp_path / "cw", [(0, "k_copy", "WRITE_SIZE", 1024.0)])
    text = ps.summary_traffic(str(tmp_path / "fetch"), str(tmp_path / "write"), str(tmp_path / "cf"),
                              str(tmp_path / "cw"), 1 << 20, "w", ["cmd"], {"grid": 1})
    rec = json.loads(text.split("traffic-json: ")[1])
    fam = rec["per_dispatch"]["k_level"]
    assert abs(fam["read_bytes"] - 2 * 1024 * (5 * 10.0 + 70.0) / 6) < 1e-6
    assert abs(fam["write_bytes"] - 1024 * (5 * 1.0 + 7.0) / 6) < 1e-6
    assert set(rec["per_dispatch"]) == {"k_level"}
