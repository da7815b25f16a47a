"""Batched solves: many uneven 1D periodic instances advanced together.

Workload: 512 instances, n log-uniform in [2^10, 2^16], tau0 ~ U[0.005, 0.5],
Q_T ~ U[0, 3], one acoustic mode m ~ U{1..16} of amplitude 1e-3, 10000 steps
each.  Every instance has its own dt (eq. (16)); all advance in one step kernel
per step.

Measured (``measure``):
  batch_fp32, batch_mixed, batch_fp64
      the whole batch in FP32 (FP32 deviation state, FP64 totals), mixed
      (FP32 arithmetic, FP64 deviation state) and FP64: GPU seconds, solves/s,
      cell-updates/s.  The FP32 batch takes 10000 steps per instance; the
      others run each instance to the FP32 batch's end time of that instance
      (within a step or so of 10000 steps), so all states compare at equal
      times.
  one_at_a_time_fp64
      each instance alone on the GPU in FP64, one after another: the wall time
      per step of a sample of instances, extrapolated to the whole workload
      (labelled so).
  accuracy (every instance)
      the decay or growth rate of the acoustic mode fitted per instance from
      snapshots, in each precision; the FP64 discretisation error of that rate
      estimated from a second FP64 batch on grids of n // 2 cells (Richardson:
      |r(n) - r(n')| / ((n/n')^2 - 1)); an instance is at equal accuracy in a
      precision when that precision's rate differs from the FP64 rate by no
      more than the FP64 discretisation error.  Also the relative L1 error of
      the final perturbation against FP64 at equal time.
  speedup
      solves/s of each batched precision over one-at-a-time FP64, and the
      number of instances at equal accuracy in that precision.

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


def mode_amplitude(U: np.ndarray, nx: int, rho0: float, mode: int) -> complex:
    """Complex Fourier coefficient of the density perturbation at the mode."""
    x = wl.cell_centres(nx)
    k = 2.0 * math.pi * mode
    return complex(np.sum((U[0, 0] - rho0) * np.exp(-1j * k * x)) * 2.0 / nx)


def fit_rate(ts, amps) -> float:
    """Slope of log |amplitude| against time (least squares)."""
    ts, amps = np.asarray(ts), np.abs(np.asarray(amps))
    return float(np.polyfit(ts, np.log(amps), 1)[0])


def perturbation_error(U: np.ndarray, ref: np.ndarray) -> float:
    """Largest over components of sum |U - ref| / sum |ref - mean(ref)|, over
    the components whose perturbation is not zero; raises on a NaN."""
    errs = []
    for q in range(ref.shape[0]):
        den = float(np.abs(ref[q] - ref[q].mean()).sum())
        if not den > 0.0:
            continue
        errs.append(float(np.abs(U[q] - ref[q]).sum()) / den)
    if not errs or any(not math.isfinite(e) for e in errs):
        raise FloatingPointError(f"perturbation error undefined: {errs}")
    return max(errs)


def run_batch(torch, insts, prec, steps, snapshots, t_ends=None, refine_down=False):
    """All instances in one batch: ``steps`` steps each, or (t_ends given) each
    instance to its own end time.  Returns the GPU seconds of the steps, per
    instance the snapshot times and mode amplitudes, the final states and
    final times.  refine_down: grids of n // 2 cells (same modes)."""
    grids = [(i["nx"] // 2 if refine_down else i["nx"]) for i in insts]
    Ws = [wl.acoustic_mode_1d(i["gas"], n, i["mode"], 1e-3) if refine_down else i["W"]
          for i, n in zip(insts, grids)]
    arena = int(sum(ng.Batch.solve_bytes(n, 1, prec) for n in grids) * 1.05) + (256 << 20)
    b = ng.Batch(len(insts), arena, precision=prec)
    if t_ends is None:
        slots = [b.add(i["gas"], n, 1, W, t_end=1e30, max_steps=steps)
                 for i, n, W in zip(insts, grids, Ws)]
        total = steps
    else:
        slots = [b.add(i["gas"], n, 1, W, t_end=te, max_steps=4 * steps)
                 for i, n, W, te in zip(insts, grids, Ws, t_ends)]
        total = 4 * steps
    assert all(s is not None for s in slots)
    seg = max(1, steps // snapshots) if not refine_down else max(1, steps // (2 * snapshots))

    def snap():
        for j, (s, i, n) in enumerate(zip(slots, insts, grids)):
            ts[j].append(b.diagnostics(s)["t"])
            amps[j].append(mode_amplitude(b.conserved(s), n, i["gas"]["rho0"], i["mode"]))

    ts = [[] for _ in insts]
    amps = [[] for _ in insts]
    snap()
    run_s = 0.0
    done = 0
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    while b.active() > 0 and done < total:
        k = seg
        torch.cuda.synchronize()
        ev0.record()
        b.run(k)
        ev1.record()
        torch.cuda.synchronize()
        run_s += ev0.elapsed_time(ev1) * 1e-3
        done += k
        snap()
    assert b.active() == 0, "batch did not finish"
    finals = [b.conserved(s) for s in slots]
    diags = [b.diagnostics(s) for s in slots]
    b.close()
    assert all(d["status"] == 0 for d in diags), "a batch instance failed"
    return dict(run_s=run_s, ts=ts, amps=amps, finals=finals,
                t_final=[d["t"] for d in diags], steps=[d["steps"] for d in diags])


def one_at_a_time_fp64(torch, insts, sample_count, steps_each, total_steps):
    """FP64 alone on the GPU, one instance after another, on every
    len(insts)/sample_count-th instance for steps_each steps: the mean wall
    time per step, extrapolated to total_steps steps of every instance."""
    sample = list(range(0, len(insts), max(1, len(insts) // sample_count)))[:sample_count]
    per_step = []
    for j in sample:
        i = insts[j]
        s = ng.Solver(i["gas"], i["nx"], 1, W=i["W"], precision=ng.NG_FP64)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(steps_each)
        torch.cuda.synchronize()
        per_step.append((time.perf_counter() - t0) / steps_each)
        s.close()
    t_est = float(np.mean(per_step)) * total_steps * len(insts)
    return {"solves_per_s_extrapolated": len(insts) / t_est, "seconds_extrapolated": t_est,
            "sample": f"{len(sample)} of {len(insts)} instances x {steps_each} steps alone in "
                      f"FP64 (one solve on the GPU at a time): mean wall time per step x "
                      f"{total_steps} steps x {len(insts)} instances"}


def measure(torch, count=512, steps=10000, snapshots=5, fp64_sample=32, fp64_steps=1000):
    insts = wl.batch_1d_instances(count, steps=steps)
    cells = float(sum(i["nx"] for i in insts))
    log(f"[batch] {len(insts)} instances, {cells:.3e} cells per step")
    out = {"workload": f"batch_{len(insts)}x1d_n2^10..2^16_{steps}steps",
           "instances": len(insts), "steps_each": steps, "cells_per_step": cells}
    log("[batch] one at a time in FP64 (sample)")
    solo = one_at_a_time_fp64(torch, insts, fp64_sample, fp64_steps, steps)
    out["one_at_a_time_fp64"] = solo
    runs = {}
    log("[batch] fp32 batch")
    runs["fp32"] = run_batch(torch, insts, ng.NG_FP32, steps, snapshots)
    t_end = runs["fp32"]["t_final"]
    for name, prec in (("mixed", ng.NG_MIXED), ("fp64", ng.NG_FP64)):
        log(f"[batch] {name} batch to the FP32 end times")
        runs[name] = run_batch(torch, insts, prec, steps, snapshots, t_ends=t_end)
    log("[batch] fp64 batch on n // 2 cells (discretisation error)")
    coarse = run_batch(torch, insts, ng.NG_FP64, steps, snapshots, t_ends=t_end,
                       refine_down=True)
    rates = {nm: [fit_rate(t, a) for t, a in zip(r["ts"], r["amps"])] for nm, r in runs.items()}
    r_coarse = [fit_rate(t, a) for t, a in zip(coarse["ts"], coarse["amps"])]
    disc = []
    for i, r64, rc in zip(insts, rates["fp64"], r_coarse):
        ratio = (i["nx"] / (i["nx"] // 2)) ** 2
        disc.append(abs(r64 - rc) / (ratio - 1.0))
    for name in ("fp32", "mixed", "fp64"):
        r = runs[name]
        sps = len(insts) / r["run_s"]
        rec = {"gpu_seconds": r["run_s"], "solves_per_s": sps,
               "cell_updates_per_s": float(sum(i["nx"] * n for i, n in zip(insts, r["steps"])))
               / r["run_s"],
               "steps_total": int(sum(r["steps"])),
               "speedup_vs_one_at_a_time_fp64": sps / solo["solves_per_s_extrapolated"]}
        if name != "fp64":
            rate_err = [abs(a - b) for a, b in zip(rates[name], rates["fp64"])]
            pert = [perturbation_error(U, U64) for U, U64 in
                    zip(r["finals"], runs["fp64"]["finals"])]
            ok = sum(1 for e, d in zip(rate_err, disc) if e <= d)
            rec["accuracy_vs_fp64_batch"] = {
                "instances": len(insts),
                "instances_at_equal_accuracy": ok,
                "rate_error_max": max(rate_err),
                "rate_error_median": float(np.median(rate_err)),
                "fp64_rate_discretisation_error_median": float(np.median(disc)),
                "final_perturbation_rel_l1_max": max(pert),
                "final_perturbation_rel_l1_median": float(np.median(pert))}
        out[f"batch_{name}"] = rec
        log(f"[batch] {name}: {rec}")
    # the speedup at equal accuracy is claimed only for a precision whose
    # every instance is at equal accuracy
    eq = {nm: out[f"batch_{nm}"]["accuracy_vs_fp64_batch"]["instances_at_equal_accuracy"]
          == len(insts) for nm in ("fp32", "mixed")}
    out["equal_accuracy_on_every_instance"] = eq
    best = [nm for nm in ("fp32", "mixed") if eq[nm]]
    out["speedup_at_equal_accuracy"] = (
        {"precision": max(best, key=lambda nm: out[f"batch_{nm}"]["solves_per_s"]),
         "value": max(out[f"batch_{nm}"]["speedup_vs_one_at_a_time_fp64"] for nm in best)}
        if best else None)
    out["batched_fp64_speedup_vs_one_at_a_time_fp64"] = \
        out["batch_fp64"]["speedup_vs_one_at_a_time_fp64"]
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--count", type=int, default=512)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--snapshots", type=int, default=5)
    ap.add_argument("--fp64-sample", type=int, default=32)
    ap.add_argument("--fp64-steps", type=int, default=1000)
    args = ap.parse_args(argv)
    import torch
    assert torch.cuda.is_available()
    ng.lib()
    out = measure(torch, args.count, args.steps, args.snapshots, args.fp64_sample,
                  args.fp64_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
