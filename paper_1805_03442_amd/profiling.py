"""Summaries of rocprofv3 output for the step kernels.

``python -m paper_1805_03442_amd.profiling stats <kernel_stats.csv> --command ...``
    markdown table of per-kernel durations (``--kernel-trace --stats``);
``python -m paper_1805_03442_amd.profiling counters <counter_collection.csv> ...``
    mean per dispatch of every counter of one kernel (e.g. the SQ_ instruction
    counts);
``python -m paper_1805_03442_amd.profiling traffic <fetch.csv> <write.csv> ...``
    HBM bytes per launch of one kernel from a ``--pmc FETCH_SIZE`` and a
    ``--pmc WRITE_SIZE`` run (KiB per dispatch), each scaled by what the same
    counter reads for a device-to-device copy of known size in the same run.

The traffic record is written as JSON text with the hash of the kernel sources
it was measured on; bench.py reports it only while that hash still matches.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import statistics
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNEL_SOURCES = ["paper_1805_03442_amd/csrc/ng_kernels.hip",
                  "paper_1805_03442_amd/csrc/ng_cell.hpp",
                  "paper_1805_03442_amd/csrc/ng_csph.hpp",
                  "paper_1805_03442_amd/csrc/ng_internal.hpp"]


def kernel_hash(root: str = ROOT) -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(root, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def stats_markdown(path: str, command: str, top: int = 12, bench_json: str | None = None,
                   leg: str | None = None) -> str:
    rows = list(csv.DictReader(open(path)))
    out = [f"Command: `{command}`", "",
           "| kernel | calls | mean us | min us | max us | share |",
           "|---|---|---|---|---|---|"]
    for r in rows[:top]:
        name = r["Name"].replace("|", "/")
        if len(name) > 90:
            name = name[:87] + "..."
        out.append(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                   f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | "
                   f"{float(r['Percentage']):.1f}% |")
    if bench_json:
        # the benchmark's own line from the same run: its HIP-event kernel
        # duration is the figure the profiler's mean above should match
        with open(bench_json) as f:
            line = [ln for ln in f if ln.startswith("{")][-1]
        b = json.loads(line)
        if leg:
            # a leg of the benchmark with a roofline of its own
            b = b[leg]
            b = dict(b, ms_per_step=b["us_per_step"] * 1e-3)
        r = b["roofline"]
        out += ["", f"Same run, bench.py's own measurement: `{r['kernel']}` mean "
                f"{1e3 * r['kernel_ms']:.1f} us over the timed launches (HIP events carried by "
                f"each launch), {b['ms_per_step'] * 1e3:.1f} us per step, value "
                f"{b['value']:.3e} {b['unit']}."]
    out += ["", f"Kernel source hash: {kernel_hash()}"]
    return "\n".join(out) + "\n"


def _per_dispatch(path: str):
    rows = list(csv.DictReader(open(path)))
    out = []
    for r in rows:
        out.append(dict(name=r["Kernel_Name"], grid=int(r["Grid_Size"]),
                        value=float(r["Counter_Value"]), counter=r["Counter_Name"],
                        dur=int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
    return out


def traffic(fetch_csv: str, write_csv: str, kernel: str, copy_bytes: int, alg_bytes: float):
    """Bytes per launch of ``kernel`` (substring of the kernel name)."""
    res = {}
    for tag, path in (("fetch", fetch_csv), ("write", write_csv)):
        d = _per_dispatch(path)
        # calibration: the copies are the largest copyBuffer dispatches
        copies = [x for x in d if "copyBuffer" in x["name"]]
        copies.sort(key=lambda x: x["value"], reverse=True)
        cal = [x["value"] for x in copies[:3]]
        kib_copy = statistics.mean(cal)
        # a device-to-device copy reads and writes copy_bytes
        factor = (copy_bytes / 1024.0) / kib_copy
        ks = [x["value"] for x in d if kernel in x["name"]]
        res[tag] = dict(kib_per_launch=statistics.mean(ks), launches=len(ks),
                        copy_kib=kib_copy, factor=factor,
                        bytes_per_launch=statistics.mean(ks) * 1024.0 * factor)
    total = res["fetch"]["bytes_per_launch"] + res["write"]["bytes_per_launch"]
    return dict(kernel=kernel, bytes_per_launch=total, algorithmic_bytes=alg_bytes,
                ratio=total / alg_bytes, fetch=res["fetch"], write=res["write"],
                kernel_hash=kernel_hash())


def counters_by_name(path: str, kernel: str) -> dict:
    by = {}
    for x in _per_dispatch(path):
        if kernel in x["name"]:
            by.setdefault(x["counter"], []).append(x["value"])
    return by


def counters_markdown(path: str, kernel: str, command: str) -> str:
    by = counters_by_name(path, kernel)
    out = [f"Command: `{command}`", "", f"Kernel: `{kernel}`", "",
           "| counter | dispatches | mean per dispatch |", "|---|---|---|"]
    for c in sorted(by):
        out.append(f"| {c} | {len(by[c])} | {statistics.mean(by[c]):.6g} |")
    out += ["", f"Kernel source hash: {kernel_hash()}"]
    return "\n".join(out) + "\n"


def coop_markdown(trace_csv: str, command: str, specs: list, bench_json: str | None) -> str:
    """Per-step times of cooperative launches from a kernel trace.  specs:
    "name-part:steps:workgroups:label" -- the longest launch of a kernel whose
    name holds name-part with that many workgroups ran `steps` steps."""
    rows = list(csv.DictReader(open(trace_csv)))
    out = [f"Command: `{command}`", "",
           "| run | kernel | workgroups x threads | launch us | steps | us per step |",
           "|---|---|---|---|---|---|"]
    for spec in specs:
        part, steps, groups, label = spec.split(":", 3)
        best = None
        for r in rows:
            g = int(r["Grid_Size_X"]) // int(r["Workgroup_Size_X"])
            if part in r["Kernel_Name"] and g == int(groups):
                d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
                if best is None or d > best[0]:
                    best = (d, r)
        if best is None:
            raise SystemExit(f"no launch of {part} with {groups} workgroups")
        d, r = best
        name = r["Kernel_Name"].split("(")[0].replace("void ", "")
        out.append(f"| {label} | `{name}` | {groups} x {r['Workgroup_Size_X']} | {d:.1f} | "
                   f"{steps} | {d / int(steps):.2f} |")
    if bench_json:
        with open(bench_json) as f:
            b = json.loads([ln for ln in f if ln.startswith("{")][-1])
        p1 = b.get("periodic_1d_2e20", {})
        ac = b.get("acoustic_1d_1024", {})
        figs = [f"{k} {p1[k]['us_per_step']:.2f}" for k in ("fp32", "fp64", "mixed") if k in p1]
        out += ["", "Same run, bench.py's own measurement (HIP events around the call that "
                "takes the steps): 2^20 cells "
                + ", ".join(figs) + " us per step"
                + (f"; 1024 cells FP64 {ac['us_per_step']:.2f} us per step" if ac else "") + "."]
    out += ["", f"Kernel source hash: {kernel_hash()}"]
    return "\n".join(out) + "\n"


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("csv")
    a.add_argument("--command", required=True)
    a.add_argument("--out", required=True)
    a.add_argument("--bench-json", default=None,
                   help="stdout of the profiled bench.py run (its JSON line)")
    a.add_argument("--leg", default=None,
                   help="key of the benchmark leg whose roofline the summary quotes")
    b = sub.add_parser("traffic")
    b.add_argument("fetch_csv")
    b.add_argument("write_csv")
    b.add_argument("--kernel", default="step2d_kernel<ng::Dev32<5>")
    b.add_argument("--copy-bytes", type=int, default=1 << 30)
    b.add_argument("--alg-bytes", type=float, default=40.0 * 4096 * 4096)
    b.add_argument("--command", required=True)
    b.add_argument("--out-json", required=True)
    b.add_argument("--out-md", required=True)
    d = sub.add_parser("coop")
    d.add_argument("trace_csv")
    d.add_argument("--command", required=True)
    d.add_argument("--out", required=True)
    d.add_argument("--bench-json", default=None)
    d.add_argument("--launch", action="append", required=True,
                   help="name-part:steps:workgroups:label of a cooperative run")
    c = sub.add_parser("counters")
    c.add_argument("csv")
    c.add_argument("--kernel", default="step2d_kernel<ng::Dev32<5>")
    c.add_argument("--command", required=True)
    c.add_argument("--out", required=True)
    c.add_argument("--out-json", default=None)
    args = ap.parse_args(argv)
    if args.cmd == "counters":
        md = counters_markdown(args.csv, args.kernel, args.command)
        with open(args.out, "w") as f:
            f.write(md)
        if args.out_json:
            by = counters_by_name(args.csv, args.kernel)
            rec = dict(kernel=args.kernel, command=args.command, kernel_hash=kernel_hash(),
                       mean_per_dispatch={k: statistics.mean(v) for k, v in by.items()})
            with open(args.out_json, "w") as f:
                json.dump(rec, f, indent=1)
        print(md)
        return
    if args.cmd == "coop":
        md = coop_markdown(args.trace_csv, args.command, args.launch, args.bench_json)
        with open(args.out, "w") as f:
            f.write(md)
        print(md)
        return
    if args.cmd == "stats":
        md = stats_markdown(args.csv, args.command, bench_json=args.bench_json, leg=args.leg)
        with open(args.out, "w") as f:
            f.write(md)
        print(md)
        return
    rec = traffic(args.fetch_csv, args.write_csv, args.kernel, args.copy_bytes, args.alg_bytes)
    rec["command"] = args.command
    with open(args.out_json, "w") as f:
        json.dump(rec, f, indent=1)
    md = [f"Command (one pass per counter): `{args.command}`", "",
          f"Kernel: `{args.kernel}`", "",
          "| counter | KiB/launch | copy KiB (1 GiB D2D) | scale | bytes/launch |",
          "|---|---|---|---|---|"]
    for tag, name in (("fetch", "FETCH_SIZE"), ("write", "WRITE_SIZE")):
        r = rec[tag]
        md.append(f"| {name} | {r['kib_per_launch']:.0f} | {r['copy_kib']:.0f} | "
                  f"{r['factor']:.3f} | {r['bytes_per_launch'] / 1e6:.1f} MB |")
    md += ["", f"Total HBM traffic {rec['bytes_per_launch'] / 1e6:.1f} MB per launch against "
           f"{rec['algorithmic_bytes'] / 1e6:.1f} MB algorithmic ({rec['ratio']:.2f}x).",
           f"Kernel source hash: {rec['kernel_hash']}"]
    with open(args.out_md, "w") as f:
        f.write("\n".join(md) + "\n")
    print("\n".join(md))


if __name__ == "__main__":
    main(sys.argv[1:])
