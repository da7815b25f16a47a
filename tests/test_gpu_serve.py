"""GPU test of the continuous-batching server: requests of different sizes,
gases and end times arrive while others run; each served result is bitwise the
result of the same solve run alone, and latency statistics are recorded."""
import numpy as np
import pytest

from paper_1805_03442_amd import workloads as wl

pytestmark = pytest.mark.gpu


def small_trace(count=12):
    recs = wl.serve_trace(count=count, rate=20000.0, log2_1d=(8.0, 11.0), side_2d=(32.0, 96.0),
                          t_end=(0.005, 0.02))
    return recs


def test_served_results_equal_alone_runs():
    import torch
    from paper_1805_03442_amd import ng, serve
    assert torch.cuda.is_available()
    recs = small_trace()
    reqs = serve.requests_from_trace(recs, wl.request_state)
    budget = sum(ng.Batch.solve_bytes(r.nx, r.ny) for r in reqs) // 2 + (64 << 20)
    be = serve.GpuBackend(capacity=6, budget_bytes=budget, keep_results=True)
    srv = serve.Server(be, capacity=6, tick_steps=16)
    st = srv.run_trace(reqs, max_wall=120.0)
    print("serve stats", st, flush=True)
    assert st["completed"] == len(reqs)
    assert st["resident_max"] >= 2
    assert st["p50_latency_s"] <= st["p99_latency_s"]
    for r in srv.stats.completed:
        s = ng.Solver(r.gas, r.nx, r.ny, W=r.state(), precision=ng.NG_FP32)
        s.run_to_time(r.t_end)
        U = s.conserved()
        assert s.diagnostics()["steps"] == r.steps
        s.close()
        assert np.array_equal(U, r.result), (r.id, r.nx, r.ny)
    be.close()
