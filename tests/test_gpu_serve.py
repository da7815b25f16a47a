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


def _perturbation_rel_l1(U, ref, U0, comps):
    """Largest over components of sum |U - ref| / sum |ref - U0| (components
    with a non-zero change only)."""
    errs = []
    for q in comps:
        den = float(np.abs(ref[q] - U0[q]).sum())
        if den > 0.0:
            errs.append(float(np.abs(U[q] - ref[q]).sum()) / den)
    assert errs and all(np.isfinite(errs))
    return max(errs)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_served_results_match_the_oracle(prec):
    """Requests of mixed 1D/2D sizes, gases and end times, admitted while
    others run (capacity 5, half the arena they would need at once), against
    the oracle running each one alone to the same end time: FP64 bit for bit
    with the same number of steps; FP32 within 1e-5 relative L1 of the change
    of the state (runs of 6 to 120 steps, long before shocks)."""
    import torch
    import oracle
    from paper_1805_03442_amd import ng, serve
    assert torch.cuda.is_available()
    oracle.build()
    precision = ng.NG_FP64 if prec == "fp64" else ng.NG_FP32
    recs = small_trace(10)
    reqs = serve.requests_from_trace(recs, wl.request_state)
    budget = sum(ng.Batch.solve_bytes(r.nx, r.ny, precision) for r in reqs) // 2 + (64 << 20)
    be = serve.GpuBackend(capacity=5, budget_bytes=budget, precision=precision,
                          keep_results=True)
    srv = serve.Server(be, capacity=5, tick_steps=16)
    st = srv.run_trace(reqs, max_wall=120.0)
    print("serve stats", st, flush=True)
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert st["resident_max"] >= 2
    for r in srv.stats.completed:
        c = [0, 1, 3, 4] if r.ny == 1 else [0, 1, 2, 3, 4]
        P = oracle.Problem(r.gas, r.nx, r.ny)
        U0 = P.prim_to_cons(r.state())
        ref = P.run(U0, 10 ** 7, t_end=r.t_end)
        assert ref["status"] == 0
        print(f"request {r.id} {r.nx}x{r.ny} steps {r.steps} oracle {ref['steps']}", flush=True)
        if prec == "fp64":
            assert r.steps == ref["steps"]
            assert np.array_equal(r.result[c], ref["U"][c]), (r.id, r.nx, r.ny)
        else:
            assert abs(r.steps - ref["steps"]) <= 1
            e = _perturbation_rel_l1(r.result, ref["U"], U0, c)
            print(f"  fp32 perturbation rel L1 {e:.2e}", flush=True)
            assert e <= 1e-5, (r.id, r.nx, r.ny, e)
    be.close()
