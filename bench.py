#!/usr/bin/env python3
"""Throughput of the fused FP32 MUSCL step on a 2D periodic 4096 x 4096 grid.

One step = one pass of the whole hot path over the grid: primitive recovery,
limited slopes, half-step predictor, HLLC face fluxes, sources, the
conservative update of eq. (15), the signal-speed maximum for the next dt of
eq. (16), FP64 totals and source budgets, and the per-solve reduction that
accepts the step and advances t.

Timing: at least 0.3 s of warm-up steps (and at least --warmup steps), then
five windows of --steps steps, each between HIP events on the solver's stream;
``value`` and ``ms_per_step`` come from the median window.  One more window of
max(--steps, 100) steps launches every step kernel with its own start and end
events; their mean is the kernel duration of ``roofline``.

Prints one JSON line:
  value       cell-updates/s of the median window (state resident in HBM)
  roofline    the step kernel's algorithmic bytes per launch (40 B per cell:
              read 5 FP32 planes, write 5) over its mean launch time, against
              the 8 TB/s HBM peak; traffic from the committed rocprofv3
              FETCH_SIZE/WRITE_SIZE summary when it was taken on the current
              kernel source, else null; "alu": vector lane-operations per second
              (committed SQ_INSTS_VALU count x 64 over the same launch time)
              against the non-packed FP32 issue peak, the limit this kernel
              actually runs into
  config3_5000_steps  the workload's whole run (5000 steps) in FP32, FP64 and
              mixed (FP32 arithmetic on an FP64 deviation state): wall time,
              cell-updates/s, the step kernels' durations (one extra window),
              and the FP32 and mixed errors against FP64 at the same end time
  batch       512 uneven 1D instances: FP32, mixed and FP64 batches against one
              solve at a time in FP64, equal accuracy checked on every instance
  served      the served stream (continuous batching): scaled sizes to the end
              (p50/p99 latency, solves/s) and the full sizes for a bounded
              wall time (completed, backlog, offered load)
  bounded_ends  the FP32 step on the same grid with wall and outflow ends
  periodic_1d_2e20  the 1D 2^20-cell multi-mode run (20000 steps) in FP32,
              FP64 and mixed on the cooperative path (FP32 also with one
              launch per step), with the FP32 / mixed error against FP64
  acoustic_1d_1024  the 1024-cell FP64 acoustic run (2000 steps) on the GPU,
              cooperative and in the one-workgroup persistent kernel
  forced_source_1d, sector_2d, blast_waves_1d  section 3's runs (1D also at
              102400 cells) and section 2.4's blast waves at 128000 cells,
              in FP32 and FP64 with the FP32 error against FP64
  csph_1d     the CSPH-TVD step (section 2.3) in FP64 on a 2^22-cell periodic
              grid: cell-updates/s, its roofline (vector ALU issue and HBM),
              the oracle on two whole steps; and section 2.4's blast waves
              (figure 2) on 200 and 1600 cells with CSPH-TVD and MUSCL
  cpu_baseline  the serial FP64 oracle on whole steps of the same grid (about
              10 s of one host core), the host CPU model, and batch_fleet: the
              512-instance 1D batch workload's sample on the oracle in one
              process per host core (aggregate rate, solves/s extrapolated),
              and per_config_1d: the two 1D workloads on one core
Input: seeded synthetic isotropic k^-2 density field (|k| <= 64, rms 1e-3),
isentropic pressure, fluid at rest; gas of eqs. (1)-(7) with Q_T = 2.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_CELL_FP32 = 40.0   # 5 conserved planes read + 5 written, 4 B each
BYTES_PER_CELL_FP64 = 80.0
BYTES_PER_CELL_CSPH = 64.0   # 1D: 4 FP64 conserved planes read + 4 written
CSPH_VALU_FILE = os.path.join(ROOT, "profiles", "step1d_csph_fp64_4m_valu.txt")
CSPH_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "step1d_csph_fp64_4m_traffic.txt")
CSPH_KERNEL = "step1d_kernel<ng::Plain64<4>, 4>"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "step2d_fp32_4096_traffic.txt")
VALU_FILE = os.path.join(ROOT, "profiles", "step2d_fp32_4096_valu.txt")
# non-packed FP32 vector issue of MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
# (the published 157.3 TFLOP/s counts a packed FMA as 4 flops per lane-cycle)
VALU_PEAK_TLANEOPS = 256 * 4 * 16 * 2.4e9 / 1e12


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def counter_record(path):
    """A committed rocprofv3 counter summary, if it was taken on the current
    kernel source."""
    from paper_1805_03442_amd.profiling import kernel_hash
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_hash") != kernel_hash():
        return None
    return rec


def traffic_record():
    """Measured HBM bytes per launch of the step kernel."""
    return counter_record(TRAFFIC_FILE)


WARMUP_SECONDS = 0.3
REPS = 5


# steps per captured HIP graph (ng_set_graph_steps); --no-graphs sets the
# library's largest value, 4096, which no call of the timed legs reaches
# (they issue at most a few hundred steps per call), so that every step is a
# direct launch (counter passes of rocprofv3 run that way)
GRAPH_STEPS = None
NO_GRAPH_STEPS = 4096


def setup_solver(s):
    from paper_1805_03442_amd import autotune
    autotune.apply(s)
    if GRAPH_STEPS is not None:
        s.set_graph_steps(GRAPH_STEPS)


def timed_run(ng, torch, gas, W, n, steps, warmup, precision, bc=(0, 0, 0, 0), reps=REPS,
              ny=None, tune=True, coop=None, **kw):
    """Warm-up (>= WARMUP_SECONDS and >= warmup steps), ``reps`` windows of
    ``steps`` steps between HIP events on the solver's stream (median), then
    one window of max(steps, 100) steps whose every step kernel carries its
    own start/end events (mean kernel duration).  ny: n x n when None; kw go
    to the solver (riemann, scheme); tune: apply the cached launch shape;
    coop: ng_set_coop's cell limit (0: one launch per step for a 1D solve)."""
    s = ng.Solver(gas, n, n if ny is None else ny, W=W, precision=precision, bc=bc, **kw)
    if tune:
        setup_solver(s)
    elif GRAPH_STEPS is not None:
        s.set_graph_steps(GRAPH_STEPS)
    if coop is not None:
        s.set_coop(coop)
    st = torch.cuda.current_stream()
    s.step(max(warmup, 1))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    warm = max(warmup, 1)
    while time.perf_counter() - t0 < WARMUP_SECONDS:
        s.step(20)
        torch.cuda.synchronize()
        warm += 20
    wins = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(st)
        s.step(steps)
        e1.record(st)
        torch.cuda.synchronize()
        wins.append(e0.elapsed_time(e1))
    kw = max(steps, 100)
    s.enable_timing(kw, 1)
    s.step(kw)
    torch.cuda.synchronize()
    step_ms, fin_ms, launches = s.kernel_time()
    s.enable_timing(0, 1)
    d = s.diagnostics()
    s.close()
    assert d["status"] == 0, d
    med = sorted(wins)[len(wins) // 2]
    return dict(total_ms=med, windows_ms=wins, warmup_steps=warm, step_ms=step_ms,
                fin_ms=fin_ms, launches=launches, diag=d)


def run_whole(ng, torch, gas, W, n, precision, steps=None, t_end=None):
    """A whole run (steps, or to t_end) through ng_step / ng_run_to_time
    between HIP events, then one window of 50 steps with every step kernel
    timed; returns the state at the end of the run and the rates."""
    s = ng.Solver(gas, n, n, W=W, precision=precision)
    setup_solver(s)
    s.step(1)
    torch.cuda.synchronize()
    d0 = s.diagnostics()
    st = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(st)
    if t_end is None:
        s.step(steps - 1)
    else:
        s.run_to_time(t_end)
    e1.record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    d = s.diagnostics()
    assert d["status"] == 0, d
    U = s.conserved()
    taken = d["steps"] - d0["steps"]
    s.enable_timing(50, 1)
    s.step(50)
    torch.cuda.synchronize()
    kms, _, _ = s.kernel_time()
    s.close()
    return dict(U=U, t=d["t"], steps=d["steps"], run_ms=ms, wall_s=wall,
                cell_updates_per_s=float(n) * n * taken / (ms * 1e-3), step_kernel_ms=kms)


def host_cpu():
    """Model name of the host CPU and the number of cores this process may use."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return dict(model=model, cores_available=len(os.sched_getaffinity(0)))


def cpu_baseline(gas, W, n, min_seconds=10.0, max_steps=8):
    """The serial FP64 oracle on whole steps of the same grid (dt of eq. (16)
    and the update), repeated until about ``min_seconds`` of CPU work."""
    import oracle
    oracle.build()
    P = oracle.Problem(gas, n, n)
    U = P.prim_to_cons(W)
    steps, el = 0, 0.0
    while steps < max_steps and el < min_seconds:
        t0 = time.perf_counter()
        dt = P.dt(U)
        st, U, _ = P.step(U, dt)
        el += time.perf_counter() - t0
        assert st == 0
        steps += 1
    return dict(value=steps * n * n / el, unit="cell-updates/s", cores=1, kind="oracle",
                sample=f"{steps} full steps (dt from eq. (16) + the update) of the {n}x{n} "
                       f"grid, serial FP64 C oracle on one host core, {el:.1f} s",
                host=host_cpu())


def oracle_1d_configs():
    """The oracle on the two 1D workloads: the 1024-cell acoustic run whole
    (2000 steps), the 2^20-cell multi-mode run for 10 steps (its rate, and the
    20000-step run's time extrapolated from it)."""
    import oracle
    from paper_1805_03442_amd import workloads as wl
    oracle.build()
    res = {}
    for w, steps in ((wl.workload_1d_acoustic(), None), (wl.workload_1d_multimode(), 10)):
        k = w["steps"] if steps is None else steps
        P = oracle.Problem(w["gas"], w["nx"], 1)
        U = P.prim_to_cons(w["W"])
        t0 = time.perf_counter()
        r = P.run(U, k)
        el = time.perf_counter() - t0
        assert r["status"] == 0 and r["steps"] == k
        rate = w["nx"] * k / el
        res[w["name"]] = dict(value=rate, unit="cell-updates/s", cores=1, steps_timed=k,
                              seconds=el, run_seconds_extrapolated=w["nx"] * w["steps"] / rate
                              if steps is not None else None)
    return res


def _oracle_instance(task):
    """Worker of cpu_fleet: one batch instance on the serial FP64 oracle."""
    import oracle
    gas, nx, W, steps = task
    P = oracle.Problem(gas, nx, 1)
    U = P.prim_to_cons(W)
    t0 = time.perf_counter()
    r = P.run(U, steps)
    el = time.perf_counter() - t0
    assert r["status"] == 0 and r["steps"] == steps
    return nx * steps, el


def cpu_fleet(count=512, steps_each=10000, every=8, steps=400, max_workers=16):
    """The batch workload (count uneven 1D instances, steps_each steps each) on
    the serial FP64 oracle, one process per host core: every ``every``-th
    instance for ``steps`` steps, the processes fed largest first; aggregate
    cell-updates/s over the wall time, and the whole workload's solves/s
    extrapolated from it.  Runs before anything touches the GPU (the worker
    processes are forked)."""
    import multiprocessing as mp
    import oracle
    from paper_1805_03442_amd import workloads as wl
    oracle.build()
    insts = wl.batch_1d_instances(count, steps=steps_each)
    sample = sorted(insts[::every], key=lambda i: -i["nx"])
    workers = max(1, min(max_workers, len(os.sched_getaffinity(0))))
    tasks = [(i["gas"], i["nx"], i["W"], steps) for i in sample]
    with mp.get_context("fork").Pool(workers) as pool:
        t0 = time.perf_counter()
        res = pool.map(_oracle_instance, tasks, chunksize=1)
        wall = time.perf_counter() - t0
    done = float(sum(r[0] for r in res))
    rate = done / wall
    total = float(sum(i["nx"] for i in insts)) * steps_each
    return dict(value=rate, unit="cell-updates/s", cores=workers, kind="oracle",
                solves_per_s_extrapolated=count / (total / rate),
                sample=f"{len(sample)} of the {count} batch instances (every {every}th) x "
                       f"{steps} steps, one serial FP64 oracle process per core, {wall:.1f} s "
                       f"wall; solves/s extrapolated to {count} instances x {steps_each} steps")


def error_vs(U, ref, U0, names):
    """Relative L1 of the full field and of the change from U0, per component."""
    import numpy as np
    full, pert = {}, {}
    for c, nm in names:
        full[nm] = float(np.abs(U[c] - ref[c]).sum() / np.abs(ref[c]).sum())
        den = float(np.abs(ref[c] - U0[c]).sum())
        pert[nm] = float(np.abs(U[c] - ref[c]).sum() / den) if den > 0 else None
    return {"rel_l1": full, "rel_l1_of_perturbation": pert}


def csph_leg(ng, torch, np, wl, args, fine_rho=None):
    """The CSPH-TVD step of section 2.3 (1D, FP64, HLL): throughput on the
    2^22-cell periodic workload on the per-step path (timed windows, then
    every step kernel timed by its own events), its roofline (vector ALU
    issue from the committed SQ_INSTS_VALU count of the kernel, and HBM at
    64 algorithmic bytes per cell), the paper's figure-2 runs (blast waves
    between walls to t = 0.038 on 200 and 1600 cells, CSPH-TVD beside MUSCL,
    L1 density difference from the 128000-cell MUSCL run when that leg ran)
    and section 3's forced-source runs with both schemes (skipped with the
    paper's other runs), and the oracle on two whole steps of the same grid
    on one host core."""
    wc = wl.workload_csph_1d()
    nc = wc["nx"]
    k = args.csph_steps
    log(f"[bench] CSPH-TVD 1D {nc} cells: {REPS} windows of {k} steps")
    # one launch per step (the cooperative path would take this grid too, at
    # about the same rate: 2^22 cells are compute-bound either way), so that
    # the timed kernel is the step kernel whose roofline is reported
    r = timed_run(ng, torch, wc["gas"], wc["W"], nc, k, args.warmup, ng.NG_FP64, ny=1,
                  tune=False, coop=0, riemann=ng.NG_HLL, scheme=ng.NG_CSPH_TVD)
    value = nc * k / (r["total_ms"] * 1e-3)
    kern_s = r["step_ms"] * 1e-3
    hbm = BYTES_PER_CELL_CSPH * nc / kern_s / 1e9
    roof = {"bound": "alu", "kernel": CSPH_KERNEL, "kernel_ms": r["step_ms"],
            "launches_timed": r["launches"], "finalize_ms": r["fin_ms"],
            "hbm": {"achieved": hbm, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": hbm / HBM_PEAK_GBS,
                    "algorithmic_bytes_per_launch": BYTES_PER_CELL_CSPH * nc}}
    vr = counter_record(CSPH_VALU_FILE)
    if vr is not None and "SQ_INSTS_VALU" in vr["mean_per_dispatch"]:
        insts = vr["mean_per_dispatch"]["SQ_INSTS_VALU"]
        ach = insts * 64 / kern_s / 1e12
        roof.update({"achieved": ach, "peak": VALU_PEAK_TLANEOPS, "unit": "T lane-op/s",
                     "frac": ach / VALU_PEAK_TLANEOPS, "valu_insts_per_launch": insts,
                     "lane_ops_per_cell_update": insts * 64 / nc})
        m = vr["mean_per_dispatch"]
        if "SQ_ACTIVE_INST_VALU" in m and "GRBM_GUI_ACTIVE" in m:
            roof["valu_busy"] = m["SQ_ACTIVE_INST_VALU"] * 4 / 1024 / (m["GRBM_GUI_ACTIVE"] / 8)
    else:
        roof.update({"achieved": None, "peak": VALU_PEAK_TLANEOPS, "unit": "T lane-op/s",
                     "frac": None})
    tr = counter_record(CSPH_TRAFFIC_FILE)
    roof["hbm"]["traffic"] = tr["bytes_per_launch"] if tr is not None else None
    res = {"workload": wc["name"], "precision": "fp64", "riemann": "hll", "steps": k,
           "path": "one launch per step",
           "value": value, "unit": "cell-updates/s", "us_per_step": 1e3 * r["total_ms"] / k,
           "windows_ms": r["windows_ms"], "roofline": roof}
    log(f"[bench] CSPH-TVD {value:.3e} cell-updates/s, step kernel {1e3 * r['step_ms']:.1f} us")
    if not args.no_cpu_baseline:
        import oracle
        oracle.build()
        P = oracle.CsphProblem(wc["gas"], nc)
        U0 = P.prim_to_cons(wc["W"])
        t0 = time.perf_counter()
        ref = P.run(U0, 2)
        el = time.perf_counter() - t0
        assert ref["status"] == 0
        res["cpu_baseline"] = {"value": nc * 2 / el, "unit": "cell-updates/s", "cores": 1,
                               "kind": "oracle", "sample": f"2 whole steps of the {nc}-cell grid"}
    if args.no_source_runs:
        return res
    # figure 2: blast waves, CSPH-TVD and MUSCL on the same grids
    gb = dict(wl.BASE_GAS, Cv=0.0, tau_rho=0.0, tau_T=0.0, Q0=0.0, Q_rho=0.0, Q_T=0.0,
              I0=0.0, I_rho=0.0, I_T=0.0, tau0=1.0)
    bw = {}
    for nb in (200, 1600):
        for name, scheme, riemann in (("csph_tvd", ng.NG_CSPH_TVD, ng.NG_HLL),
                                      ("muscl", ng.NG_MUSCL, ng.NG_HLLC)):
            best = None
            for _ in range(2):      # the first run also loads the path's kernels
                s = ng.Solver(gb, nb, 1, W=wl.blast_waves_1d(nb), precision=ng.NG_FP64,
                              riemann=riemann, bc=(ng.NG_BC_WALL, ng.NG_BC_WALL, 0, 0),
                              scheme=scheme)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                taken = s.run_to_time(0.038)
                el = time.perf_counter() - t0
                rho = s.conserved()[0, 0]
                d = s.diagnostics()
                s.close()
                assert d["status"] == 0
                best = el if best is None else min(best, el)
            rec = {"steps": taken, "wall_ms": 1e3 * best, "us_per_step": 1e6 * best / taken,
                   "rho_max": float(rho.max()),
                   "x_rho_max": float((np.argmax(rho) + 0.5) / nb)}
            if fine_rho is not None:
                avg = fine_rho.reshape(nb, -1).mean(axis=1)
                rec["l1_rho_vs_muscl_128000"] = float(np.mean(np.abs(rho - avg)))
            bw[f"{name}_n{nb}"] = rec
    res["blast_waves_t0038"] = bw
    log(f"[bench] CSPH-TVD blast waves: {bw}")
    # section 3's forced-source runs to t = 0.8 with both schemes (FP64): the
    # relative L1 difference of the velocity fields at the paper's sizes and
    # at 12800 cells
    xc = {}
    for stage in ("linear", "nonlinear"):
        ws = wl.workload_forced_source(stage)
        for n in (ws["nx"], 12800):
            u, rec = {}, {}
            for name, scheme, riemann in (("csph_tvd", ng.NG_CSPH_TVD, ng.NG_HLL),
                                          ("muscl", ng.NG_MUSCL, ng.NG_HLLC)):
                s = ng.Solver(ws["gas"], n, 1, W=wl.uniform_state(ws["gas"], n),
                              precision=ng.NG_FP64, riemann=riemann, bc=ws["bc"],
                              source=ws["source"], scheme=scheme)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                taken = s.run_to_time(ws["t_end"])
                el = time.perf_counter() - t0
                U = s.conserved()
                d = s.diagnostics()
                s.close()
                assert d["status"] == 0
                u[name] = U[1, 0] / U[0, 0]
                rec[name] = {"steps": taken, "wall_ms": 1e3 * el}
            rec["rel_l1_u_csph_vs_muscl"] = float(np.abs(u["csph_tvd"] - u["muscl"]).sum()
                                                  / np.abs(u["muscl"]).sum())
            xc[f"{stage}_n{n}"] = rec
    res["forced_source_t08"] = xc
    log(f"[bench] CSPH-TVD against MUSCL, forced source: {xc}")
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--config3-steps", type=int, default=5000,
                    help="length of the whole FP32/FP64/mixed run of the 2D workload (0: skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-full-wall", type=float, default=12.0)
    ap.add_argument("--bounded-steps", type=int, default=200)
    ap.add_argument("--steps-1d", type=int, default=20000)
    ap.add_argument("--no-source-runs", action="store_true",
                    help="skip the paper's runs: section 3's forced-source runs (1D and the "
                         "2D sector) and section 2.4's blast waves (MUSCL and CSPH-TVD)")
    ap.add_argument("--csph-steps", type=int, default=200,
                    help="steps per timed window of the CSPH-TVD leg (0: skip)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain device copy of known size (for counter scaling)")
    ap.add_argument("--no-graphs", action="store_true",
                    help="launch every step directly (no captured graphs; for counter passes)")
    args = ap.parse_args()
    if args.no_graphs:
        global GRAPH_STEPS
        GRAPH_STEPS = NO_GRAPH_STEPS

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    fleet = None
    blast_fine_rho = None
    if not args.no_cpu_baseline:
        # before the GPU is touched: the oracle's worker processes are forked
        log("[bench] CPU fleet: the batch instances on the oracle, one process per core")
        fleet = cpu_fleet()
        log(f"[bench] oracle fleet {fleet['value']:.3e} cell-updates/s on {fleet['cores']} cores")

    import numpy as np
    import torch
    from paper_1805_03442_amd import ng, workloads as wl
    assert torch.cuda.is_available(), "needs a GPU"
    torch.cuda.set_device(0)
    ng.lib()

    n = args.n
    log(f"[bench] building the {n}x{n} synthetic input")
    gas = dict(wl.BASE_GAS, Q_T=2.0)
    W = wl.random_field_2d(gas, n, wl.rng(3))

    log(f"[bench] FP32: warmup >= {args.warmup} steps and {WARMUP_SECONDS} s, "
        f"{REPS} windows of {args.steps} steps")
    r32 = timed_run(ng, torch, gas, W, n, args.steps, args.warmup, ng.NG_FP32)
    cells = float(n) * n
    ms_per_step = r32["total_ms"] / args.steps
    value = cells * args.steps / (r32["total_ms"] * 1e-3)
    achieved = BYTES_PER_CELL_FP32 * cells / (r32["step_ms"] * 1e-3) / 1e9
    log(f"[bench] FP32 {ms_per_step:.4f} ms/step (windows {r32['windows_ms']}), step kernel "
        f"{r32['step_ms']:.4f} ms, finalize {r32['fin_ms']:.4f} ms, {value:.3e} cell-updates/s")

    tr = traffic_record()
    traffic = None
    if tr is not None:
        traffic = tr["bytes_per_launch"]

    out = {
        "metric": "cell-updates/s (FP32 fused MUSCL step, 2D 4096^2) + %HBM roofline; "
                  "p50/p99 solve latency",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"2d_periodic_{n}x{n}_random_field_fp32", "nx": n, "ny": n,
                   "precision": "fp32 deviations, fp64 totals", "riemann": "hllc",
                   "cfl": 0.4, "Q_T": 2.0},
        "timing": {"windows_ms": r32["windows_ms"], "statistic": "median of windows",
                   "warmup_steps_run": r32["warmup_steps"],
                   "warmup_seconds_min": WARMUP_SECONDS},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "step2d_kernel<Dev32<5>>",
                     "kernel_ms": r32["step_ms"], "launches_timed": r32["launches"],
                     "finalize_ms": r32["fin_ms"],
                     "algorithmic_bytes_per_launch": BYTES_PER_CELL_FP32 * cells},
    }
    # the step is limited by vector ALU issue: lane-operations per second from
    # the committed SQ_INSTS_VALU count of this kernel over the same launch time
    vr = counter_record(VALU_FILE)
    if vr is not None and "SQ_INSTS_VALU" in vr["mean_per_dispatch"]:
        insts = vr["mean_per_dispatch"]["SQ_INSTS_VALU"]
        ach = insts * 64 / (r32["step_ms"] * 1e-3) / 1e12
        out["roofline"]["alu"] = {"achieved": ach, "peak": VALU_PEAK_TLANEOPS,
                                  "unit": "T lane-op/s", "frac": ach / VALU_PEAK_TLANEOPS,
                                  "valu_insts_per_launch": insts,
                                  "lane_ops_per_cell_update": insts * 64 / cells}
        m = vr["mean_per_dispatch"]
        if "SQ_ACTIVE_INST_VALU" in m and "GRBM_GUI_ACTIVE" in m:
            # share of the kernel's cycles in which a SIMD issues VALU work:
            # 4 cycles per wave64 instruction over 1024 SIMDs, against the
            # GPU-busy cycles of one of the 8 XCDs
            out["roofline"]["alu"]["valu_busy"] = (m["SQ_ACTIVE_INST_VALU"] * 4 / 1024
                                                   / (m["GRBM_GUI_ACTIVE"] / 8))

    if args.config3_steps > 0:
        # the workload's whole run in each precision: FP32 takes the steps, FP64
        # and mixed run to the FP32 end time (the same time within their own
        # dt sequence), so the errors compare states at equal time
        k = args.config3_steps
        log(f"[bench] 2D {n}^2: the whole {k}-step run in FP32, FP64, mixed")
        res = {}
        runs = {}
        runs["fp32"] = run_whole(ng, torch, gas, W, n, ng.NG_FP32, steps=k)
        for name, prec in (("fp64", ng.NG_FP64), ("mixed", ng.NG_MIXED)):
            runs[name] = run_whole(ng, torch, gas, W, n, prec, t_end=runs["fp32"]["t"])
        s0 = ng.Solver(gas, n, n, W=W, precision=ng.NG_FP64)
        U0 = s0.conserved()
        s0.close()
        names = list(enumerate(["rho", "rho_u", "rho_v", "E", "E_nu"]))
        for name in ("fp32", "fp64", "mixed"):
            r = runs[name]
            bpc = BYTES_PER_CELL_FP32 if name == "fp32" else BYTES_PER_CELL_FP64
            res[name] = {"steps": r["steps"], "t_end": r["t"], "run_ms": r["run_ms"],
                         "cell_updates_per_s": r["cell_updates_per_s"],
                         "step_kernel_ms": r["step_kernel_ms"],
                         "hbm_frac": bpc * cells / (r["step_kernel_ms"] * 1e-3) / 1e9
                         / HBM_PEAK_GBS}
            if name != "fp64":
                res[name]["vs_fp64"] = error_vs(r["U"], runs["fp64"]["U"], U0, names)
            log(f"[bench] config 3 {name}: {res[name]}")
        # the shock indicator of the parity definitions: smallest ratio of
        # neighbouring pressures along x and y
        Wf = runs["fp64"]["U"]
        rho = Wf[0]
        p = 0.4 * (Wf[3] - 0.5 * (Wf[1] ** 2 + Wf[2] ** 2) / rho - Wf[4])
        rx = np.minimum(p / np.roll(p, -1, 1), np.roll(p, -1, 1) / p).min()
        ry = np.minimum(p / np.roll(p, -1, 0), np.roll(p, -1, 0) / p).min()
        res["min_neighbour_pressure_ratio"] = float(min(rx, ry))
        out["config3_5000_steps"] = dict(res, workload=f"2d_random_{n}x{n}", steps=k)
        del runs, Wf, rho, p

    if not args.no_batch:
        from paper_1805_03442_amd import bench_batch
        log("[bench] batch of 512 uneven 1D instances")
        out["batch"] = bench_batch.measure(torch)

    if not args.no_serve:
        from paper_1805_03442_amd import bench_serve
        budget = 200 << 30
        log("[bench] served stream, scaled sizes, to the end")
        recs = wl.serve_trace(count=400, log2_1d=(10.0, 14.0), side_2d=(64.0, 256.0),
                              t_end=(0.005, 0.02))
        sc = bench_serve.run(recs, budget, 1024, 32, 120.0)
        log(f"[bench] served scaled: {sc}")
        log(f"[bench] served stream, full sizes, {args.serve_full_wall} s")
        recs = wl.serve_trace(count=2000)
        fu = bench_serve.run(recs, budget, 1024, 32, args.serve_full_wall)
        log(f"[bench] served full: {fu}")
        out["served"] = {
            "budget_bytes": budget, "capacity": 1024, "tick_steps": 32,
            "scaled": dict(sc, trace="400 requests, Poisson 200/s, 1D n 2^10..2^14, "
                                     "2D 64^2..256^2, t_end 0.005..0.02, run to the end"),
            "full": dict(fu, trace="2000 requests, Poisson 200/s, 1D n 2^12..2^20, "
                                   "2D 256^2..2048^2, t_end 0.1..2, "
                                   f"{args.serve_full_wall} s of wall time")}

    if args.steps_1d > 0:
        # 1D periodic 2^20 cells, 64 random modes, Q_T = 2: the whole run of
        # steps_1d steps in each precision (the library's path for a lone 1D
        # solve: one cooperative launch with a grid barrier per step; FP32
        # also with one graph-launched kernel per step, for comparison), and
        # the FP32 / mixed error against FP64 at the end
        k = args.steps_1d
        w1 = wl.workload_1d_multimode()
        n1 = w1["nx"]
        res1, fin1 = {}, {}

        def run_1d(prec, coop):
            s = ng.Solver(w1["gas"], n1, 1, W=w1["W"], precision=prec)
            setup_solver(s)
            if not coop:
                s.set_coop(0)
            s.step(20)
            torch.cuda.synchronize()
            st = torch.cuda.current_stream()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(st)
            s.step(k)
            e1.record(st)
            torch.cuda.synchronize()
            U = s.conserved()
            s.close()
            return e0.elapsed_time(e1), U

        for name, prec in (("fp32", ng.NG_FP32), ("fp64", ng.NG_FP64), ("mixed", ng.NG_MIXED)):
            ms, fin1[name] = run_1d(prec, True)
            res1[name] = {"value": n1 * k / (ms * 1e-3), "unit": "cell-updates/s",
                          "us_per_step": 1e3 * ms / k, "path": "cooperative"}
            log(f"[bench] 1D 2^20 {name}: {res1[name]['value']:.3e} cell-updates/s")
        ms, U = run_1d(ng.NG_FP32, False)
        assert np.array_equal(U, fin1["fp32"])
        res1["fp32"]["us_per_step_one_launch_per_step"] = 1e3 * ms / k
        s0 = ng.Solver(w1["gas"], n1, 1, W=w1["W"], precision=ng.NG_FP64)
        U0 = s0.conserved()
        s0.close()
        for name in ("fp32", "mixed"):
            res1[name]["rel_l1_of_perturbation_vs_fp64"] = max(
                float(np.abs(fin1[name][c] - fin1["fp64"][c]).sum()
                      / np.abs(fin1["fp64"][c] - U0[c]).sum()) for c in (0, 1, 3, 4))
        out["periodic_1d_2e20"] = dict(res1, steps=k + 20, workload=w1["name"])

    if args.steps_1d > 0:
        # the 1024-cell acoustic mode in FP64, its whole run of 2000 steps (one
        # cooperative launch over 5 CUs; a first run loads the kernel), and
        # the same run in the persistent one-workgroup kernel
        w0 = wl.workload_1d_acoustic()
        for rep in range(3):
            s = ng.Solver(w0["gas"], w0["nx"], 1, W=w0["W"], precision=ng.NG_FP64)
            if rep == 2:
                s.set_coop(0)
                ms_coop = ms
            torch.cuda.synchronize()
            st = torch.cuda.current_stream()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(st)
            s.step(w0["steps"])
            e1.record(st)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            s.close()
        out["acoustic_1d_1024"] = {"workload": w0["name"], "precision": "fp64",
                                   "steps": w0["steps"], "run_ms": ms_coop,
                                   "us_per_step": 1e3 * ms_coop / w0["steps"],
                                   "value": w0["nx"] * w0["steps"] / (ms_coop * 1e-3),
                                   "unit": "cell-updates/s", "path": "cooperative",
                                   "us_per_step_one_workgroup": 1e3 * ms / w0["steps"]}
        log(f"[bench] 1D 1024 FP64 acoustic run: {ms_coop:.2f} ms for {w0['steps']} steps "
            f"(one workgroup: {ms:.2f} ms)")

    if args.bounded_steps > 0:
        # the same grid between reflecting walls (x) and outflow ends (y):
        # ghost cells from the boundary rules instead of wrap-around
        k = args.bounded_steps
        log(f"[bench] FP32 with wall/outflow ends: timing {k} steps")
        rb = timed_run(ng, torch, gas, W, n, k, 5, ng.NG_FP32,
                       bc=(ng.NG_BC_WALL, ng.NG_BC_WALL, ng.NG_BC_OUTFLOW, ng.NG_BC_OUTFLOW),
                       reps=3)
        out["bounded_ends"] = {"bc": "x walls, y outflow", "steps": k,
                               "value": cells * k / (rb["total_ms"] * 1e-3),
                               "unit": "cell-updates/s", "step_kernel_ms": rb["step_ms"],
                               "hbm_frac": BYTES_PER_CELL_FP32 * cells / (rb["step_ms"] * 1e-3)
                               / 1e9 / HBM_PEAK_GBS}

    if not args.no_source_runs:
        # section 3's 1D runs: sound from a source at x = 0 into the unstable
        # medium to t = 0.8 (linear stage S = 0.5, N = 800; shock train S = 1,
        # N = 1600), each precision to the end, and the FP32 / mixed error of
        # the final perturbation against FP64
        res = {}
        for stage, nfine in (("linear", None), ("nonlinear", None), ("nonlinear", 102400)):
            ws = wl.workload_forced_source(stage)
            key = stage
            if nfine:
                # the paper's 10^5-cell reference size
                ws = dict(ws, nx=nfine, W=wl.uniform_state(ws["gas"], nfine),
                          name=ws["name"].rsplit("_n", 1)[0] + f"_n{nfine}")
                key = f"{stage}_n{nfine}"
            fin, rec = {}, {}
            for name, prec in (("fp64", ng.NG_FP64), ("fp32", ng.NG_FP32),
                               ("mixed", ng.NG_MIXED)):
                s = ng.Solver(ws["gas"], ws["nx"], 1, W=ws["W"], precision=prec, bc=ws["bc"],
                              source=ws["source"])
                if prec == ng.NG_FP64:
                    Ub = s.conserved()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                taken = s.run_to_time(ws["t_end"])
                el = time.perf_counter() - t0
                fin[name] = s.conserved()
                d = s.diagnostics()
                s.close()
                assert d["status"] == 0
                rec[name] = {"steps": taken, "wall_ms": 1e3 * el,
                             "cell_updates_per_s": ws["nx"] * taken / el}
            W64 = fin["fp64"]
            rho = W64[0, 0]
            u = W64[1, 0] / rho
            jumps = np.abs(np.diff(rho))
            amp = ws["source"][0]
            smooth = amp * 2 * math.pi / ws["source"][1] / ws["nx"]
            for name in ("fp32", "mixed"):
                rec[name]["rel_l1_of_perturbation_vs_fp64"] = max(
                    float(np.abs(fin[name][c] - W64[c]).sum() / np.abs(W64[c] - Ub[c]).sum())
                    for c in (0, 1, 3, 4))
            steep = jumps > 5 * smooth
            res[key] = dict(rec, workload=ws["name"], t_end=ws["t_end"],
                            max_abs_u=float(np.abs(u).max()),
                            shock_faces=int(steep.sum()),
                            # runs of consecutive steep faces: one per shock
                            shocks=int(steep[0] + (steep[1:] & ~steep[:-1]).sum()))
            log(f"[bench] forced source {key}: {res[key]}")
        out["forced_source_1d"] = res

        # section 2.4's blast waves between walls to t = 0.038 at the paper's
        # reference size (128000 cells, ~514000 steps) in FP64 and FP32
        gb = dict(wl.BASE_GAS, Cv=0.0, tau_rho=0.0, tau_T=0.0, Q0=0.0, Q_rho=0.0, Q_T=0.0,
                  I0=0.0, I_rho=0.0, I_T=0.0, tau0=1.0)
        nb = 128000
        fin, rec = {}, {}
        for name, prec in (("fp64", ng.NG_FP64), ("fp32", ng.NG_FP32)):
            s = ng.Solver(gb, nb, 1, W=wl.blast_waves_1d(nb), precision=prec,
                          bc=(ng.NG_BC_WALL, ng.NG_BC_WALL, 0, 0))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            taken = s.run_to_time(0.038)
            el = time.perf_counter() - t0
            fin[name] = s.conserved()
            d = s.diagnostics()
            s.close()
            assert d["status"] == 0
            rec[name] = {"steps": taken, "wall_ms": 1e3 * el,
                         "cell_updates_per_s": nb * taken / el}
        blast_fine_rho = fin["fp64"][0, 0]
        rec["fp32"]["rel_l1_vs_fp64"] = {
            nm: float(np.abs(fin["fp32"][c] - fin["fp64"][c]).sum()
                      / np.abs(fin["fp64"][c]).sum())
            for c, nm in ((0, "rho"), (1, "rho_u"), (3, "E"))}
        out["blast_waves_1d"] = dict(rec, workload=f"blast_waves_walls_n{nb}", t_end=0.038)
        log(f"[bench] blast waves: {out['blast_waves_1d']}")

        # the 2D sector run of section 3 (active 30-degree wedge from the
        # source, wall G1, free flow G2-G4) to t = 1 in FP32 and FP64: the
        # wave's amplitude inside and outside the wedge, the FP32 error
        ws = wl.workload_sector_2d()
        fin, rec = {}, {}
        for name, prec in (("fp64", ng.NG_FP64), ("fp32", ng.NG_FP32)):
            s = ng.Solver(ws["gas"], ws["nx"], ws["ny"], W=ws["W"], h=ws["h"], precision=prec,
                          bc=ws["bc"], source=ws["source"], wedge=ws["wedge"])
            setup_solver(s)
            if prec == ng.NG_FP64:
                Ub = s.conserved()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            taken = s.run_to_time(ws["t_end"])
            el = time.perf_counter() - t0
            fin[name] = s.conserved()
            d = s.diagnostics()
            s.close()
            assert d["status"] == 0
            rec[name] = {"steps": taken, "wall_ms": 1e3 * el,
                         "cell_updates_per_s": ws["nx"] * ws["ny"] * taken / el}
        rec["fp32"]["rel_l1_of_perturbation_vs_fp64"] = {
            nm: float(np.abs(fin["fp32"][c] - fin["fp64"][c]).sum()
                      / np.abs(fin["fp64"][c] - Ub[c]).sum())
            for c, nm in enumerate(["rho", "rho_u", "rho_v", "E", "E_nu"])}
        drho = np.abs(fin["fp64"][0] - Ub[0])
        act = ws["active"]
        out["sector_2d"] = dict(rec, workload=ws["name"], t_end=ws["t_end"],
                                max_drho_in_wedge=float(drho[act].max()),
                                max_drho_outside=float(drho[~act].max()))
        log(f"[bench] sector: {out['sector_2d']}")

    if args.csph_steps > 0:
        out["csph_1d"] = csph_leg(ng, torch, np, wl, args, blast_fine_rho)

    if args.calibrate_copy:
        nbytes = 1 << 30
        a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"[bench] copy calibration: 3 copies of {nbytes} bytes")

    if not args.no_cpu_baseline:
        log("[bench] CPU baseline: oracle steps of the full grid")
        out["cpu_baseline"] = cpu_baseline(gas, W, n)
        out["cpu_baseline"]["batch_fleet"] = fleet
        out["cpu_baseline"]["per_config_1d"] = oracle_1d_configs()
        log(f"[bench] oracle {out['cpu_baseline']['value']:.3e} cell-updates/s")

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
