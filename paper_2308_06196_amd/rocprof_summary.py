"""Summaries of rocprofv3 output for the stage kernels (kernel traces and counters).

Reads the CSV files that `rocprofv3 --output-format csv -d DIR -o run` writes:

  DIR/run_kernel_stats.csv        (--kernel-trace --stats)
  DIR/run_kernel_trace.csv        (--kernel-trace)
  DIR/run_counter_collection.csv  (--pmc ...)

Subcommands:

  stats DIR [--steps N]    print the kernel table (calls, average us, share) and,
                           from the trace, the kernel time per RK3 step of each
                           storage precision against the wall time those steps span
                           (over the last N steps of each precision when given)
  counters DIR             per-launch averages of every collected counter over the
                           stage kernels (k_stage*, first launches excluded)
  traffic --out FILE --copy-fetch DIR --copy-write DIR --entry KEY FETCH_DIR WRITE_DIR ...
                           HBM bytes per stage launch from FETCH_SIZE and WRITE_SIZE
                           passes, each scaled by the factor the same counter reads
                           for a plain device copy of known size (bench.py
                           --copy-probe), written with the kernel sources' hash
"""
from __future__ import annotations

import argparse
import csv
import json
import os
import re
import sys
from collections import defaultdict

STAGE = re.compile(r"k_stage")


def _rows(path):
    with open(path, newline="") as fh:
        yield from csv.DictReader(fh)


def short(name: str) -> str:
    """void bgk::k_stage<2, 3, double, 0, false>(bgk::StageArgs) -> k_stage<2,3,double,0,false>"""
    m = re.search(r"(k_\w+(?:<[^>]*>)?)", name)
    return m.group(1).replace(" ", "") if m else name


def kernel_stats(d):
    out = []
    for r in _rows(os.path.join(d, "run_kernel_stats.csv")):
        out.append({"kernel": short(r["Name"]), "calls": int(r["Calls"]),
                    "avg_us": float(r["AverageNs"]) / 1e3, "pct": float(r["Percentage"])})
    return out


def kernel_trace(d):
    out = []
    for r in _rows(os.path.join(d, "run_kernel_trace.csv")):
        out.append({"kernel": short(r["Kernel_Name"]), "start": int(r["Start_Timestamp"]),
                    "end": int(r["End_Timestamp"])})
    out.sort(key=lambda r: r["start"])
    return out


def step_times(d, last_steps=0):
    """Per storage precision (from the stage kernels' type): kernel time per RK3
    step (stage + equilibrium launches between the first and last stage launch of
    that precision) and the wall time those launches span, both in ms per step.
    last_steps > 0 keeps only the last that many steps of each precision (the
    timed steps of a benchmark run, after its warm-up steps)."""
    tr = kernel_trace(d)
    res = {}
    groups = defaultdict(list)
    for i, r in enumerate(tr):
        k = r["kernel"]
        if k.startswith("k_stage"):
            args = k[k.index("<") + 1:-1].split(",")
            key = "bf16" if args[-1] == "true" else ("fp64" if "double" in args else "fp32")
            groups[key].append(i)
    for key, idx in groups.items():
        if last_steps:
            idx = idx[-3 * last_steps:]
        lo, hi = idx[0], idx[-1]
        # the equilibrium solve launched just before the first stage belongs to it
        while lo > 0 and tr[lo - 1]["kernel"].startswith("k_newton"):
            lo -= 1
        seg = tr[lo:hi + 1]
        busy = sum(r["end"] - r["start"] for r in seg)
        span = seg[-1]["end"] - seg[0]["start"]
        steps = len(idx) / 3.0
        stage = [tr[i]["end"] - tr[i]["start"] for i in idx]
        res[key] = {"stage_launches": len(idx), "stage_avg_us": sum(stage) / len(stage) / 1e3,
                    "kernel_ms_per_step": busy / steps / 1e6, "span_ms_per_step": span / steps / 1e6}
    return res


def counters(d, skip_first=0):
    """{kernel: {counter: mean per launch}} over launches of the stage kernels."""
    per = defaultdict(lambda: defaultdict(float))
    names = {}
    for r in _rows(os.path.join(d, "run_counter_collection.csv")):
        k = short(r["Kernel_Name"])
        if not STAGE.search(k):
            continue
        per[int(r["Dispatch_Id"])][r["Counter_Name"]] += float(r["Counter_Value"])
        names[int(r["Dispatch_Id"])] = k
    disp = sorted(per)[skip_first:]
    out = defaultdict(lambda: defaultdict(list))
    for i in disp:
        for c, v in per[i].items():
            out[names[i]][c].append(v)
    return {k: {c: sum(v) / len(v) for c, v in cs.items()} | {"launches": len(next(iter(cs.values())))}
            for k, cs in out.items()}


def launches(d, counter):
    """Per stage launch (dispatch order): the counter's value summed over its instances."""
    per = defaultdict(float)
    for r in _rows(os.path.join(d, "run_counter_collection.csv")):
        if STAGE.search(r["Kernel_Name"]) and r["Counter_Name"] == counter:
            per[int(r["Dispatch_Id"])] += float(r["Counter_Value"])
    return [per[i] for i in sorted(per)]


def copy_factor(d, counter, nbytes=1 << 30):
    """bytes / (KiB the counter reads) for the 1 GiB device copy of bench.py --copy-probe."""
    vals = []
    for r in _rows(os.path.join(d, "run_counter_collection.csv")):
        if r["Counter_Name"] == counter and "copy" in r["Kernel_Name"].lower():
            vals.append(float(r["Counter_Value"]))
    if not vals:  # the copy kernel's name varies; take the largest dispatch
        per = defaultdict(float)
        for r in _rows(os.path.join(d, "run_counter_collection.csv")):
            if r["Counter_Name"] == counter:
                per[int(r["Dispatch_Id"])] += float(r["Counter_Value"])
        vals = [max(per.values())]
    kib = sorted(vals)[len(vals) // 2]
    return nbytes / 1024.0 / kib


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    a1 = sub.add_parser("stats")
    a1.add_argument("dir")
    a1.add_argument("--steps", type=int, default=0,
                    help="per-step figures over the last STEPS steps of each precision")
    a2 = sub.add_parser("counters")
    a2.add_argument("dir")
    a3 = sub.add_parser("traffic")
    a3.add_argument("--out", required=True)
    a3.add_argument("--copy-fetch", required=True)
    a3.add_argument("--copy-write", required=True)
    a3.add_argument("--entry", nargs=3, action="append", metavar=("KEY", "FETCH_DIR", "WRITE_DIR"),
                    required=True)
    a = ap.parse_args(argv)
    if a.cmd == "stats":
        print("| kernel | calls | avg us | % |")
        print("|---|---|---|---|")
        for r in kernel_stats(a.dir):
            print(f"| {r['kernel']} | {r['calls']} | {r['avg_us']:.1f} | {r['pct']:.1f} |")
        for k, v in step_times(a.dir, a.steps).items():
            print(f"{k}: {v['stage_launches']} stage launches, average {v['stage_avg_us']:.1f} us; "
                  f"kernel time {v['kernel_ms_per_step']:.3f} ms per step within "
                  f"{v['span_ms_per_step']:.3f} ms per step of wall time")
    elif a.cmd == "counters":
        print(json.dumps(counters(a.dir), indent=1))
    else:
        sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
        import bench
        ff = copy_factor(a.copy_fetch, "FETCH_SIZE")
        fw = copy_factor(a.copy_write, "WRITE_SIZE")
        out = {"source_hash": bench.kernel_source_hash(), "fetch_factor": ff, "write_factor": fw}
        for key, fd, wd in a.entry:
            f = launches(fd, "FETCH_SIZE")
            w = launches(wd, "WRITE_SIZE")
            fb = sum(f) / len(f) * 1024.0 * ff
            wb = sum(w) / len(w) * 1024.0 * fw
            out[key] = {"bytes_per_launch": fb + wb, "fetch_bytes": fb, "write_bytes": wb,
                        "fetch_per_launch_KiB_raw": [round(x, 1) for x in f],
                        "write_per_launch_KiB_raw": [round(x, 1) for x in w]}
        with open(a.out, "w") as fh:
            json.dump(out, fh, indent=1)
        print(json.dumps({k: (v["bytes_per_launch"] if isinstance(v, dict) else v)
                          for k, v in out.items()}, indent=1))


if __name__ == "__main__":
    main()
