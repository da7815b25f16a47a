"""Launch-shape autotuner for the step kernels.

The step kernels take two shape parameters (``ng_set_launch``): rows per work
item (2D: rows a wavefront marches through; 1D: 60-cell segments per work
item) and wavefronts per workgroup.  Every cell's arithmetic is the same for
all shapes, so tuning never changes results (only the summation order of the
FP64 totals).  The tuner times each candidate with HIP events on a throwaway
solve of the target shape and caches the winner per (dimension, precision,
size bucket) in ``tuning.json`` next to this file.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np

from . import ng
from . import workloads as wl

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")

CANDIDATES = {
    2: [(r, w) for r in (4, 8, 16, 24, 32, 48, 64) for w in (1, 2, 4)],
    1: [(s, w) for s in (1, 2, 4, 8, 16, 32) for w in (1, 2, 4)],
}


def bucket(n: int) -> int:
    return int(2 ** round(math.log2(max(int(n), 1))))


def key(nx: int, ny: int, precision: int) -> str:
    dim = 1 if ny == 1 else 2
    p = {ng.NG_FP32: "fp32", ng.NG_FP64: "fp64", ng.NG_MIXED: "mixed"}[precision]
    return f"{dim}d_{p}_{bucket(nx)}x{bucket(ny)}"


def load_cache(path: str = CACHE) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def lookup(nx: int, ny: int, precision: int, path: str = CACHE):
    """(rows, waves) tuned for this shape's bucket, else None: the library's
    automatic per-solve shape (rows or segments per item chosen from the grid
    size) then applies."""
    cache = load_cache(path)
    e = cache.get(key(nx, ny, precision))
    if e is None:
        return None
    return e["rows"], e["waves"]


def apply(solver: "ng.Solver", path: str = CACHE) -> bool:
    """Set a solver's launch shape from the cache; False when nothing fits."""
    lw = lookup(solver.nx, solver.ny, solver.num.precision, path)
    if lw is None:
        return False
    solver.set_launch(*lw)
    return True


def tune(nx: int, ny: int, precision: int, gas: dict | None = None, W=None, steps: int = 30,
         warmup: int = 5, candidates=None, path: str | None = CACHE, verbose: bool = False):
    """Time every candidate shape on a throwaway solve; cache and return the
    fastest as dict(rows, waves, step_ms, table)."""
    import torch
    gas = dict(gas or dict(wl.BASE_GAS, Q_T=2.0))
    if W is None:
        r = np.random.Generator(np.random.PCG64(12345))
        if ny == 1:
            W = wl.multimode_1d(gas, nx, r, nmodes=8, kmax=max(2, min(64, nx // 8)))
        else:
            W = wl.random_field_2d(gas, max(nx, ny), r, kmax=max(1, min(32, nx // 8)))[:, :ny, :nx]
    dim = 1 if ny == 1 else 2
    cands = candidates or CANDIDATES[dim]
    s = ng.Solver(gas, nx, ny, W=W, precision=precision)
    table = []
    try:
        for rows, waves in cands:
            try:
                s.set_launch(rows, waves)
            except ng.NgError:
                continue
            s.enable_timing(0)
            s.step(warmup)
            torch.cuda.synchronize()
            s.enable_timing(steps)
            s.step(steps)
            st, fin, _ = s.kernel_time()
            table.append((rows, waves, st + fin))
            if verbose:
                print(f"  rows {rows:3d} waves {waves}: {1e3 * (st + fin):8.1f} us/step", flush=True)
    finally:
        s.close()
    rows, waves, ms = min(table, key=lambda t: t[2])
    res = dict(rows=rows, waves=waves, step_ms=ms, table=table)
    if path:
        cache = load_cache(path)
        cache[key(nx, ny, precision)] = dict(rows=rows, waves=waves, step_ms=ms)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    return res


def main():
    import argparse
    ap = argparse.ArgumentParser(description="tune step-kernel launch shapes")
    ap.add_argument("--shapes", default="4096x4096:fp32,4096x4096:fp64,4096x4096:mixed,"
                                        "1048576x1:fp32,1048576x1:fp64,1048576x1:mixed,"
                                        "16384x1:fp32,256x256:fp32,"
                                        "1024x1024:fp32,2048x2048:fp32")
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--out", default=CACHE, help="tuning cache to update")
    args = ap.parse_args()
    import torch
    assert torch.cuda.is_available()
    for item in args.shapes.split(","):
        shape, p = item.split(":")
        nx, ny = (int(v) for v in shape.split("x"))
        prec = {"fp32": ng.NG_FP32, "fp64": ng.NG_FP64, "mixed": ng.NG_MIXED}[p]
        print(f"[tune] {shape} {p}", flush=True)
        r = tune(nx, ny, prec, steps=args.steps, verbose=True, path=args.out)
        print(f"[tune] {shape} {p}: rows {r['rows']} waves {r['waves']} "
              f"{1e3 * r['step_ms']:.1f} us/step", flush=True)


if __name__ == "__main__":
    main()
