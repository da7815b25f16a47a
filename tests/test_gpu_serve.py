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


def test_served_stream_with_refused_and_failing_requests():
    """A request with an unphysical initial state is refused, one whose gas
    drives the pressure negative fails mid-run; both are accounted for and
    every other request is served with its alone-run result."""
    import torch
    from paper_1805_03442_amd import ng, serve
    assert torch.cuda.is_available()
    recs = small_trace(8)
    reqs = serve.requests_from_trace(recs, wl.request_state)
    bad_state = reqs[2]
    W = wl.request_state(recs[2])
    W[3].flat[5] = -1.0
    bad_state.W = W
    sink = reqs[5]
    sink.gas = dict(sink.gas, I0=20.0, I_T=0.0)
    sink.t_end = 10.0
    budget = sum(ng.Batch.solve_bytes(r.nx, r.ny) for r in reqs) + (64 << 20)
    be = serve.GpuBackend(capacity=4, budget_bytes=budget, keep_results=True)
    srv = serve.Server(be, capacity=4, tick_steps=16)
    st = srv.run_trace(reqs, max_wall=120.0)
    print("serve stats", st, flush=True)
    assert st["rejected"] == 1 and bad_state.failed
    assert st["completed"] == len(reqs) - 1 and st["failed"] == 1 and sink.failed
    for r in srv.stats.completed:
        if r is sink:
            continue
        s = ng.Solver(r.gas, r.nx, r.ny, W=r.state(), precision=ng.NG_FP32)
        s.run_to_time(r.t_end)
        assert np.array_equal(s.conserved(), r.result), (r.id, r.nx, r.ny)
        s.close()
    be.close()
