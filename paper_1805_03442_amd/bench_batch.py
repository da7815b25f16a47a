"""Batched solves: many uneven 1D periodic instances advanced together.

Workload: 512 instances, n log-uniform in [2^10, 2^16], tau0 ~ U[0.005, 0.5],
Q_T ~ U[0, 3], one acoustic mode m ~ U{1..16} of amplitude 1e-3, 10000 steps
each, in FP32 (FP32 deviation state, FP64 totals) and in the mixed mode (FP32
arithmetic, FP64 deviation state).  Every instance has its own dt (eq. (16))
and all advance in one step kernel per step.

Reported (one JSON line): solves/s and cell-updates/s of the FP32 batch;
the same instances solved one at a time in FP64 on the same GPU (timed on a
sample of instances and steps, extrapolated per step and labelled so); the
FP32-vs-FP64 difference of the batch results at equal times on that sample,
beside the FP64 discretisation error of the fitted rate (grid n against 2n);
and the decay or growth rate of the acoustic mode fitted per instance from
snapshots.

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


def run_batch(torch, insts, prec, steps, snapshots):
    """All instances in one batch for ``steps`` steps; GPU time of the steps,
    and per instance the snapshot times, mode amplitudes and final state."""
    arena = int(sum(ng.Batch.solve_bytes(i["nx"], 1, prec) for i in insts) * 1.05) + (256 << 20)
    b = ng.Batch(len(insts), arena, precision=prec)
    slots = [b.add(i["gas"], i["nx"], 1, i["W"], t_end=1e30, max_steps=steps) for i in insts]
    assert all(s is not None for s in slots)
    seg = max(1, steps // snapshots)
    ts = [[0.0] for _ in insts]
    amps = [[mode_amplitude(b.conserved(s), i)] for s, i in zip(slots, insts)]
    run_s = 0.0
    done = 0
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    while done < steps:
        k = min(seg, steps - done)
        torch.cuda.synchronize()
        ev0.record()
        b.run(k)
        ev1.record()
        torch.cuda.synchronize()
        run_s += ev0.elapsed_time(ev1) * 1e-3
        done += k
        for j, (s, i) in enumerate(zip(slots, insts)):
            ts[j].append(b.diagnostics(s)["t"])
            amps[j].append(mode_amplitude(b.conserved(s), i))
        log(f"[batch] {done}/{steps} steps, {run_s:.3f} s of GPU time")
    assert b.active() == 0
    finals = [b.conserved(s) for s in slots]
    b.close()
    return run_s, ts, amps, finals


def fp64_reference(insts, j, times, refine):
    """FP64 alone on the instance's grid refined ``refine`` times, run to the
    given times: fitted rate and final state."""
    i = insts[j]
    n = i["nx"] * refine
    W = i["W"] if refine == 1 else wl.acoustic_mode_1d(i["gas"], n, i["mode"], 1e-3)
    inst = dict(i, nx=n)
    s = ng.Solver(i["gas"], n, 1, W=W, precision=ng.NG_FP64)
    a = [mode_amplitude(s.conserved(), inst)]
    for t in times[1:]:
        s.run_to_time(t)
        a.append(mode_amplitude(s.conserved(), inst))
    U = s.conserved()
    s.close()
    return fit_rate(times, a), U


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
    t64_est = float(np.mean(per_step_64)) * args.steps * len(insts)
    sps64 = len(insts) / t64_est
    out = {
        "workload": f"batch_{len(insts)}x1d_n2^10..2^16_{args.steps}steps",
        "instances": len(insts), "steps_each": args.steps, "cells_per_step": cells,
        "one_at_a_time_fp64": {"solves_per_s_extrapolated": sps64,
                               "seconds_extrapolated": t64_est,
                               "sample": f"{len(sample)} instances x {args.fp64_steps} steps, "
                                         f"mean per-step wall time x {args.steps} steps x "
                                         f"{len(insts)} instances"},
    }
    acc = sample[:args.acc_sample]
    for name, prec in (("fp32", ng.NG_FP32), ("mixed", ng.NG_MIXED)):
        log(f"[batch] {name} batch")
        run_s, ts, amps, finals = run_batch(torch, insts, prec, args.steps, args.snapshots)
        rates = [fit_rate(t, a) for t, a in zip(ts, amps)]
        # accuracy at equal times against FP64 alone; the FP64 rate on the grid
        # of twice the cells gives the discretisation error for scale
        per = []
        for j in acc:
            r1, U64 = fp64_reference(insts, j, ts[j], 1)
            r2, _ = fp64_reference(insts, j, ts[j], 2)
            U = finals[j]
            e = max(float(np.abs(U[q] - U64[q]).sum() / np.abs(U64[q] - U64[q].mean()).sum())
                    for q in range(4))
            per.append({"n": insts[j]["nx"], "perturbation_rel_l1": e,
                        "rate_vs_fp64": abs(rates[j] - r1), "fp64_rate_n_vs_2n": abs(r1 - r2)})
        sps = len(insts) / run_s
        out[f"batch_{name}"] = {
            "gpu_seconds": run_s, "solves_per_s": sps,
            "cell_updates_per_s": cells * args.steps / run_s,
            "speedup_vs_one_at_a_time_fp64": sps / sps64,
            "accuracy_at_equal_time": {
                "instances": len(per),
                "perturbation_rel_l1_max": max(x["perturbation_rel_l1"] for x in per),
                "rate_vs_fp64_max": max(x["rate_vs_fp64"] for x in per),
                "instances_with_rate_error_below_discretisation":
                    sum(1 for x in per if x["rate_vs_fp64"] <= x["fp64_rate_n_vs_2n"]),
                "per_instance": per},
            "fitted_rates": rates,
        }
    out["modes"] = [i["mode"] for i in insts]
    line = json.dumps(out)
    if args.json_out:
        with open(args.json_out, "w") as f:
            f.write(line + "\n")
    summary = json.loads(line)
    for name in ("fp32", "mixed"):
        summary[f"batch_{name}"].pop("fitted_rates")
        summary[f"batch_{name}"]["accuracy_at_equal_time"].pop("per_instance")
    summary.pop("modes")
    print(json.dumps(summary), flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
