"""Batched solves: many uneven 1D periodic instances advanced together.

Workload: 512 instances, n log-uniform in [2^10, 2^16], tau0 ~ U[0.005, 0.5],
Q_T ~ U[0, 3], one acoustic mode m ~ U{1..16} of amplitude 1e-3, 10000 steps
each, FP32 (deviation storage, FP64 totals).  Every instance has its own dt
(eq. (16)) and all advance in one step kernel per step.

Reported (one JSON line): solves/s and cell-updates/s of the FP32 batch;
the same instances solved one at a time in FP64 on the same GPU (timed on a
sample of instances and steps, extrapolated per step and labelled so); the
FP32-vs-FP64 error of the batch results on that sample; and the decay or
growth rate of the acoustic mode fitted per instance from snapshots.

``python -m paper_1805_03442_amd.bench_batch [--count 512] [--steps 10000]``
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import ng
from . import workloads as wl


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def mode_amplitude(U: np.ndarray, inst: dict) -> complex:
    """Complex Fourier coefficient of the density perturbation at the mode."""
    n = inst["nx"]
    x = wl.cell_centres(n)
    rho0 = inst["gas"]["rho0"]
    k = 2.0 * math.pi * inst["mode"]
    return complex(np.sum((U[0, 0] - rho0) * np.exp(-1j * k * x)) * 2.0 / n)


def fit_rate(ts, amps) -> float:
    ts, amps = np.asarray(ts), np.abs(np.asarray(amps))
    return float(np.polyfit(ts, np.log(amps), 1)[0])


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--count", type=int, default=512)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--snapshots", type=int, default=10)
    ap.add_argument("--fp64-sample", type=int, default=32)
    ap.add_argument("--fp64-steps", type=int, default=1000)
    ap.add_argument("--acc-sample", type=int, default=8)
    ap.add_argument("--json-out", default=None)
    args = ap.parse_args(argv)
    import torch
    assert torch.cuda.is_available()
    ng.lib()

    insts = wl.batch_1d_instances(args.count, steps=args.steps)
    cells = float(sum(i["nx"] for i in insts))
    log(f"[batch] {len(insts)} instances, {cells:.3e} cells per step")
    prec = ng.NG_FP32
    arena = int(sum(ng.Batch.solve_bytes(i["nx"], 1, prec) for i in insts) * 1.05) + (256 << 20)
    b = ng.Batch(len(insts), arena, precision=prec)
    slots = [b.add(i["gas"], i["nx"], 1, i["W"], t_end=1e30, max_steps=args.steps) for i in insts]
    assert all(s is not None for s in slots)

    # run in segments; time only the segments
    seg = max(1, args.steps // args.snapshots)
    ts = {s: [0.0] for s in slots}
    amps = {s: [mode_amplitude(b.conserved(s), i)] for s, i in zip(slots, insts)}
    run_s = 0.0
    done_steps = 0
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    while done_steps < args.steps:
        k = min(seg, args.steps - done_steps)
        torch.cuda.synchronize()
        ev0.record()
        b.run(k)
        ev1.record()
        torch.cuda.synchronize()
        run_s += ev0.elapsed_time(ev1) * 1e-3
        done_steps += k
        for s, i in zip(slots, insts):
            d = b.diagnostics(s)
            ts[s].append(d["t"])
            amps[s].append(mode_amplitude(b.conserved(s), i))
        log(f"[batch] {done_steps}/{args.steps} steps, {run_s:.3f} s of GPU time")
    assert b.active() == 0
    finals = {s: b.conserved(s) for s in slots}
    b.close()
    solves_per_s = len(insts) / run_s
    cu_per_s = cells * args.steps / run_s
    rates = {s: fit_rate(ts[s], amps[s]) for s in slots}

    # one at a time in FP64 on a sample of instances, each for fp64_steps
    sample = list(range(0, len(insts), max(1, len(insts) // args.fp64_sample)))[:args.fp64_sample]
    per_step_64 = []
    for j in sample:
        i = insts[j]
        s = ng.Solver(i["gas"], i["nx"], 1, W=i["W"], precision=ng.NG_FP64)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(args.fp64_steps)
        torch.cuda.synchronize()
        per_step_64.append((time.perf_counter() - t0) / args.fp64_steps)
        s.close()
    # accuracy: FP64 alone run to the FP32 batch's snapshot times (each lands
    # exactly on the time); states compared at equal time, rates fitted alike
    errs, rate_errs = [], []
    for j in sample[:args.acc_sample]:
        i = insts[j]
        sl = slots[j]
        s = ng.Solver(i["gas"], i["nx"], 1, W=i["W"], precision=ng.NG_FP64)
        a64 = [mode_amplitude(s.conserved(), i)]
        for t in ts[sl][1:]:
            s.run_to_time(t)
            a64.append(mode_amplitude(s.conserved(), i))
        U64 = s.conserved()
        s.close()
        U32 = finals[sl]
        c = [0, 1, 2, 3]
        errs.append(max(float(np.abs(U32[q] - U64[q]).sum()
                              / np.abs(U64[q] - U64[q].mean()).sum()) for q in c))
        r64 = fit_rate(ts[sl], a64)
        rate_errs.append(abs(rates[sl] - r64))
    t64_est = float(np.mean(per_step_64)) * args.steps * len(insts)
    out = {
        "workload": f"batch_{len(insts)}x1d_n2^10..2^16_fp32_{args.steps}steps",
        "instances": len(insts), "steps_each": args.steps, "cells_per_step": cells,
        "batch_fp32": {"gpu_seconds": run_s, "solves_per_s": solves_per_s,
                       "cell_updates_per_s": cu_per_s},
        "one_at_a_time_fp64": {"solves_per_s_extrapolated": len(insts) / t64_est,
                               "seconds_extrapolated": t64_est,
                               "sample": f"{len(sample)} instances x {args.fp64_steps} steps, "
                                         f"mean per-step wall time x {args.steps} steps x "
                                         f"{len(insts)} instances"},
        "speedup_solves_per_s": (solves_per_s) / (len(insts) / t64_est),
        "fp32_vs_fp64_at_equal_time": {
            "instances": len(errs),
            "perturbation_rel_l1_max": max(errs) if errs else None,
            "fitted_rate_abs_diff_max": max(rate_errs) if rate_errs else None,
            "fitted_rate_abs_max": max(abs(rates[slots[j]]) for j in sample[:args.acc_sample]),
        },
        "fitted_rates": {str(j): rates[slots[j]] for j in range(len(insts))},
        "modes": {str(j): insts[j]["mode"] for j in range(len(insts))},
    }
    line = json.dumps(out)
    if args.json_out:
        with open(args.json_out, "w") as f:
            f.write(line + "\n")
    summary = {k: v for k, v in out.items() if k not in ("fitted_rates", "modes")}
    print(json.dumps(summary), flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
