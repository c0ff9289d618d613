"""Markdown summaries of rocprofv3 output for the files under profiles/.

    python -m paper_2105_12415_amd.profile_summary trace DIR --workload W --command CMD
    python -m paper_2105_12415_amd.profile_summary sq DIR [DIR ...] --workload W --command CMD [--command CMD]
    python -m paper_2105_12415_amd.profile_summary traffic FETCH_DIR WRITE_DIR CALIB_FETCH_DIR CALIB_WRITE_DIR
        --workload W --command CMD ... --launch JSON --calib-bytes N

DIR is a rocprofv3 output directory (``-d``) written with ``--output-format
csv``; the CSV files are found below it whatever sub-directories the
profiler made.  Counter values are summed over the XCCs by rocprofv3; per
dispatch figures are averages over the dispatches of a kernel.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import sys
from collections import OrderedDict, defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
CLOCK_GHZ = 2.4
SIMDS = 1024


def short_name(name: str) -> str:
    """Kernel name without the anonymous namespace and the argument list."""
    n = name.replace("(anonymous namespace)::", "")
    if "(" in n and not n.startswith("void "):
        n = n[: n.index("(")]
    if n.startswith("void "):
        n = n[5:]
        if "(" in n:
            n = n[: n.index("(")]
    return n.strip()


def family(name: str) -> str:
    """Template-free kernel name (k_level<float, 4, 256, false> -> k_level)."""
    n = short_name(name)
    return n[: n.index("<")] if "<" in n else n


def find_csv(d: str, suffix: str) -> str:
    hits = sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))
    if not hits:
        raise FileNotFoundError(f"no *{suffix} below {d}")
    return hits[-1]


def read_counters(d: str):
    """{kernel: {"dispatches": n, counter: mean per dispatch}} plus launch shapes."""
    rows = list(csv.DictReader(open(find_csv(d, "counter_collection.csv"))))
    per = defaultdict(lambda: defaultdict(float))
    disp = defaultdict(set)
    shape = {}
    for r in rows:
        k = short_name(r["Kernel_Name"])
        per[k][r["Counter_Name"]] += float(r["Counter_Value"])
        disp[k].add(r["Dispatch_Id"])
        shape.setdefault(k, r)
    out = OrderedDict()
    for k in per:
        n = len(disp[k])
        out[k] = {"dispatches": n, **{c: v / n for c, v in per[k].items()}}
    return out, shape


def read_stats(d: str):
    rows = list(csv.DictReader(open(find_csv(d, "kernel_stats.csv"))))
    return [(short_name(r["Name"]), int(r["Calls"]), float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3,
             float(r["MaxNs"]) / 1e3, float(r["Percentage"])) for r in rows]


def avg_us(stats, kernel: str):
    for name, calls, avg, *_ in stats:
        if name == kernel:
            return avg
    return None


def fmt(v):
    if isinstance(v, str):
        return v
    if v == 0:
        return "0"
    if abs(v) >= 1e5 or abs(v) < 1e-2:
        return f"{v:.4g}"
    return f"{v:.4g}" if abs(v) >= 100 else f"{v:.3g}"


def header(title: str, commands):
    lines = [f"# {title}", "", "Commands (from the repository root on the GPU machine):", "", "```"]
    lines += list(commands)
    lines += ["```", ""]
    return lines


def summary_trace(d: str, workload: str, commands, per_depth=None):
    """Per-kernel statistics; with per_depth = (kernel family, L) also the
    average duration of that kernel's launches by launch index mod L (one
    launch per tree depth, in depth order)."""
    stats = read_stats(d)
    lines = header(f"Kernel trace: {workload}", commands)
    lines += ["| kernel | calls | avg us | min us | max us | % of GPU time |", "|---|---|---|---|---|---|"]
    for name, calls, avg, mn, mx, pct in stats:
        lines.append(f"| `{name}` | {calls} | {avg:.1f} | {mn:.1f} | {mx:.1f} | {pct:.2f} |")
    if per_depth:
        fam, L = per_depth
        rows = list(csv.DictReader(open(find_csv(d, "kernel_trace.csv"))))
        rows.sort(key=lambda r: int(r["Start_Timestamp"]))
        durs = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in rows
                if family(r["Kernel_Name"]) == fam]
        if durs and len(durs) % L == 0:
            avg = [sum(durs[k::L]) / len(durs[k::L]) for k in range(L)]
            lines += ["", f"Per-depth average of `{fam}` (launch d of every step):", "",
                      "| depth | " + " | ".join(str(k) for k in range(L)) + " |", "|---|" + "---|" * L,
                      "| avg us | " + " | ".join(f"{a:.1f}" for a in avg) + " |"]
    return "\n".join(lines) + "\n"


def summary_sq(dirs, workload: str, commands, trace_dir: str = None, cycles_per_valu: float = None):
    """SQ counters per dispatch (several ``--pmc`` runs merged by kernel)
    and, with the kernel trace's average durations, derived columns: VALU
    busy = SQ_INSTS_VALU x the cycles one wave64 FP32 instruction occupies a
    SIMD (from the FMA-loop microbenchmark) / (1024 SIMDs x 2.4 GHz x
    duration); SQ_ACTIVE_INST_VALU / SQ_INSTS_VALU (on MI355X the ratio is 1
    for every microbenchmark kind, whatever cycles its instructions take, so
    the counter counts instructions here, not cycles); the fraction of wave
    cycles spent waiting (SQ_WAIT_ANY / SQ_WAVE_CYCLES)."""
    merged = OrderedDict()
    for d in dirs:
        cnt, _ = read_counters(d)
        for k, v in cnt.items():
            merged.setdefault(k, {}).update(v)
    stats = read_stats(trace_dir) if trace_dir else None
    cols = sorted({c for v in merged.values() for c in v if c != "dispatches"})
    lines = header(f"SQ counters per dispatch: {workload}", commands)
    lines += ["| kernel | dispatches | " + " | ".join(cols) + " |", "|---|---|" + "---|" * len(cols)]
    for k, v in merged.items():
        lines.append(f"| `{k}` | {v['dispatches']} | " + " | ".join(fmt(v.get(c, float('nan'))) for c in cols) + " |")
    lines.append("")
    derived = OrderedDict()
    if stats:
        cpi = f"{cycles_per_valu:.2f}" if cycles_per_valu else "n/a"
        lines += [f"Derived (average durations from the kernel trace; {cpi} cycles per wave64 FP32 VALU "
                  "instruction from the FMA-loop microbenchmark):", "",
                  "| kernel | avg us | VALU instr / wave | VALU busy (instr x cycles) | "
                  "SQ_ACTIVE_INST_VALU / SQ_INSTS_VALU | waiting |",
                  "|---|---|---|---|---|---|"]
        for k, v in merged.items():
            us = avg_us(stats, k)
            if not us:
                continue
            den = SIMDS * CLOCK_GHZ * 1e9 * us * 1e-6
            iv, av = v.get("SQ_INSTS_VALU"), v.get("SQ_ACTIVE_INST_VALU")
            w = v.get("SQ_WAVES")
            d = {"avg_us": us,
                 "valu_per_wave": iv / w if iv is not None and w else None,
                 "valu_busy_issue": iv * cycles_per_valu / den if iv is not None and cycles_per_valu else None,
                 "active_per_inst": av / iv if av is not None and iv else None,
                 "waiting": (v["SQ_WAIT_ANY"] / v["SQ_WAVE_CYCLES"]
                             if v.get("SQ_WAIT_ANY") is not None and v.get("SQ_WAVE_CYCLES") else None)}
            derived[k] = d
            lines.append(f"| `{k}` | {us:.1f} | " + " | ".join(
                "n/a" if d[c] is None else f"{d[c]:.3g}" for c in
                ("valu_per_wave", "valu_busy_issue", "active_per_inst", "waiting")) + " |")
        lines.append("")
    return "\n".join(lines) + "\n", merged, derived


def summary_traffic(fetch_dir, write_dir, calib_fetch_dir, calib_write_dir, calib_bytes: int, workload: str,
                    commands, launch: dict, stats_dir: str = None, sources=None):
    fetch, _ = read_counters(fetch_dir)
    write, _ = read_counters(write_dir)
    cf, _ = read_counters(calib_fetch_dir)
    cw, _ = read_counters(calib_write_dir)

    def calib(c, name):
        # the copy kernel: the dispatch whose counter is the largest
        best = max(c.values(), key=lambda v: v.get(name, 0.0))
        return best[name]

    kib = calib_bytes / 1024.0
    f_scale = kib / calib(cf, "FETCH_SIZE")
    w_scale = kib / calib(cw, "WRITE_SIZE")
    stats = read_stats(stats_dir) if stats_dir else []
    lines = header(f"HBM traffic per dispatch: {workload}", commands)
    lines += [f"Calibration: a device-to-device copy of {calib_bytes / 2**20:.0f} MiB reads FETCH_SIZE = "
              f"{calib(cf, 'FETCH_SIZE'):.4g} KiB and writes WRITE_SIZE = {calib(cw, 'WRITE_SIZE'):.4g} KiB per "
              f"dispatch against {kib:.0f} KiB each way, so the scale factors are {f_scale:.3f} (fetch) and "
              f"{w_scale:.3f} (write).", "",
              "| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | scaled MB read | scaled MB written | avg us (trace) | GB/s |",
              "|---|---|---|---|---|---|---|---|"]
    # per family (the instantiations of one kernel, e.g. the deepest depth's
    # variant of k_level beside the others): bytes per dispatch averaged
    # over all of the family's dispatches
    per = OrderedDict()
    tot = OrderedDict()
    for k in fetch:
        fr = fetch[k].get("FETCH_SIZE", 0.0)
        wr = write.get(k, {}).get("WRITE_SIZE", 0.0)
        rb, wb = fr * 1024 * f_scale, wr * 1024 * w_scale
        us = avg_us(stats, k)
        gbs = (rb + wb) / (us * 1e-6) / 1e9 if us else float("nan")
        lines.append(f"| `{k}` | {fetch[k]['dispatches']} | {fr:.4g} | {wr:.4g} | {rb / 1e6:.2f} | {wb / 1e6:.2f} | "
                     f"{us if us else float('nan'):.1f} | {gbs:.0f} |")
        n = fetch[k]["dispatches"]
        t = tot.setdefault(family(k), [0.0, 0.0, 0])
        t[0] += rb * n
        t[1] += wb * n
        t[2] += n
    for fam, (rsum, wsum, n) in tot.items():
        per[fam] = {"read_bytes": rsum / n, "write_bytes": wsum / n}
    rec = {"source_sha256": sources_sha256(sources), "workload": workload, "launch": launch, "per_dispatch": per}
    lines += ["", "Machine-readable line (bench.py reports `roofline.traffic` from it only while the sha256 of "
              "dem_kernels.hip + dem_geom.hpp matches the source it runs):", "",
              "traffic-json: " + json.dumps(rec)]
    return "\n".join(lines) + "\n"


def sources_sha256(sources=None) -> str:
    h = hashlib.sha256()
    for s in sources or [os.path.join(HERE, "csrc", "dem_kernels.hip"), os.path.join(HERE, "csrc", "dem_geom.hpp")]:
        h.update(open(s, "rb").read())
    return h.hexdigest()


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("kind", choices=["trace", "sq", "traffic"])
    ap.add_argument("dirs", nargs="+")
    ap.add_argument("--workload", required=True)
    ap.add_argument("--command", action="append", default=[])
    ap.add_argument("--trace-dir", default=None)
    ap.add_argument("--launch", default="{}")
    ap.add_argument("--calib-bytes", type=int, default=1 << 30)
    ap.add_argument("--cycles-per-valu", type=float, default=None)
    ap.add_argument("--per-depth", default=None, help="KERNEL:L, e.g. k_level:6")
    a = ap.parse_args(argv)
    if a.kind == "trace":
        pd = None
        if a.per_depth:
            fam, L = a.per_depth.split(":")
            pd = (fam, int(L))
        sys.stdout.write(summary_trace(a.dirs[0], a.workload, a.command, pd))
    elif a.kind == "sq":
        sys.stdout.write(summary_sq(a.dirs, a.workload, a.command, a.trace_dir, a.cycles_per_valu)[0])
    else:
        f, w, cf, cw = a.dirs
        sys.stdout.write(summary_traffic(f, w, cf, cw, a.calib_bytes, a.workload, a.command, json.loads(a.launch),
                                         a.trace_dir))


if __name__ == "__main__":
    main()
