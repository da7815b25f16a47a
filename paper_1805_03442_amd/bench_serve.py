"""Served stream of solves with continuous batching (``serve.Server``).

Request stream: Poisson arrivals at 200 requests/s, half 1D and half 2D
periodic grids, gas parameters drawn per request (tau0, Q_T), end times drawn
per request, FP32 with FP64 totals, admitted under an HBM budget.

Two runs:
  full    the stream as specified (1D n log-uniform 2^12..2^20, 2D side
          256..2048, t_end in [0.1, 2]) for a fixed wall time; its offered load
          is far beyond one GPU, so the report is what completed, what is still
          running or queued, and the latency of what completed;
  scaled  the same stream with sizes and end times scaled down (1D 2^10..2^14,
          2D 64..256, t_end in [0.005, 0.02]) run to completion: p50/p99
          latency, solves/s and cell-updates/s.

The client side prepares each request's initial state on host threads up to
0.25 s before its arrival; latency is counted from arrival to completion.
Reported beside p50/p99: solves/s, the cell-updates/s of the completed solves
and of all work done (running solves included), and the host time spent
admitting (waiting for states, converting and uploading them).

``python -m paper_1805_03442_amd.bench_serve [--budget-gb 200] [--full-wall 60]``
"""
from __future__ import annotations

import argparse
import json
import math
import sys

from . import serve
from . import workloads as wl


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def offered_load(recs) -> float:
    """cell-updates the trace asks for: n * steps, steps ~ t_end / dt with dt =
    0.4 h / c, c ~ 1.18 (background sound speed), h = 1/n."""
    c = math.sqrt(1.4)
    tot = 0.0
    for r in recs:
        side = max(r["nx"], r["ny"])
        steps = r["t_end"] * c * side / 0.4
        tot += r["nx"] * r["ny"] * steps
    return tot


def run(recs, budget, capacity, tick, max_wall):
    reqs = serve.requests_from_trace(recs, wl.request_state)
    be = serve.GpuBackend(capacity=capacity, budget_bytes=budget)
    srv = serve.Server(be, capacity=capacity, tick_steps=tick, prefetch=16,
                       prefetch_threads=8)
    st = srv.run_trace(reqs, max_wall=max_wall, lookahead=0.25)
    st["state_wait_s"], st["add_s"] = be.state_s, be.add_s
    be.close()
    span = recs[-1]["arrival"] if recs else 0.0
    st["offered_cell_updates"] = offered_load(recs)
    st["offered_cell_updates_per_s"] = st["offered_cell_updates"] / span if span > 0 else None
    return st


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--budget-gb", type=float, default=200.0)
    ap.add_argument("--capacity", type=int, default=1024)
    ap.add_argument("--tick", type=int, default=32)
    ap.add_argument("--full-count", type=int, default=2000)
    ap.add_argument("--full-wall", type=float, default=60.0)
    ap.add_argument("--scaled-count", type=int, default=400)
    ap.add_argument("--scaled-wall", type=float, default=120.0)
    ap.add_argument("--skip-full", action="store_true")
    args = ap.parse_args(argv)
    import torch
    assert torch.cuda.is_available()
    budget = int(args.budget_gb * (1 << 30))
    out = {"budget_bytes": budget, "capacity": args.capacity, "tick_steps": args.tick}
    if not args.skip_full:
        log(f"[serve] full stream, {args.full_count} requests, {args.full_wall} s wall")
        recs = wl.serve_trace(count=args.full_count)
        out["full"] = run(recs, budget, args.capacity, args.tick, args.full_wall)
        log(f"[serve] full: {out['full']}")
    log(f"[serve] scaled stream, {args.scaled_count} requests")
    recs = wl.serve_trace(count=args.scaled_count, log2_1d=(10.0, 14.0), side_2d=(64.0, 256.0),
                          t_end=(0.005, 0.02))
    out["scaled"] = run(recs, budget, args.capacity, args.tick, args.scaled_wall)
    log(f"[serve] scaled: {out['scaled']}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
