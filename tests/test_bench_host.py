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
