"""GPU test of the entry point that allocates nothing (ng_step_static): one
FP64 step from caller device memory to caller device memory with the
library's static scratch, against the same step through the solver entry
points (ng_init_conserved + ng_step + ng_get_conserved), bit for bit, on two
calls in a row, the second on a smaller grid than the first (the scratch keeps
the first call's contents and must not leak into the second)."""
import ctypes as C

import numpy as np
import pytest

from paper_1805_03442_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _step_static(ng, torch, gas, nx, ny, U, t=0.0, riemann=0, bc=(0, 0, 0, 0), scheme=0,
                 source=(0.0, 0.0)):
    nc = 5 if ny > 1 else 4
    comps = [0, 1, 2, 3, 4] if ny > 1 else [0, 1, 3, 4]
    planes = np.ascontiguousarray(U[comps].reshape(nc, -1))
    din = torch.from_numpy(planes).cuda()
    dout = torch.full_like(din, float("nan"))
    d = ng.step_static(gas, nx, ny, din, dout, t=t, riemann=riemann, bc=bc, scheme=scheme,
                       source=source)
    out = np.zeros_like(U)
    out[comps] = dout.cpu().numpy().reshape(nc, ny, nx)
    return out, d


def _step_solver(ng, gas, nx, ny, U, t=0.0, riemann=0, bc=(0, 0, 0, 0), scheme=0,
                 source=(0.0, 0.0)):
    s = ng.Solver(gas, nx, ny, U=U, precision=ng.NG_FP64, riemann=riemann, bc=bc,
                  scheme=scheme, t0=t, source=source)
    s.step(1)
    V = s.conserved()
    d = s.diagnostics()
    s.close()
    return V, d


@pytest.mark.parametrize("case", ["2d_hllc_periodic", "1d_hll_walls", "1d_csph_walls",
                                  "1d_hllc_source", "1d_csph_source"])
def test_static_step_equals_solver_step(case):
    """The source cases step from t = 0.37 (section 3's forced source: the
    ghosts follow the time the call is given)."""
    import torch
    from paper_1805_03442_amd import ng
    assert torch.cuda.is_available()
    gas = dict(wl.BASE_GAS, Q_T=2.0)
    r = np.random.Generator(np.random.PCG64(31))
    scheme = ng.NG_CSPH_TVD if case.startswith("1d_csph") else ng.NG_MUSCL
    t, source = 0.0, (0.0, 0.0)
    if case == "2d_hllc_periodic":
        shapes, riemann, bc = [(300, 190), (130, 70)], 0, (0, 0, 0, 0)
    elif case.endswith("_source"):
        ws = wl.workload_forced_source("linear")
        gas, bc, source, t = ws["gas"], ws["bc"], ws["source"], 0.37
        shapes, riemann = [(6000, 1), (800, 1)], 1 if scheme == ng.NG_CSPH_TVD else 0
    else:
        shapes, riemann, bc = [(70000, 1), (5000, 1)], 1, (1, 1, 0, 0)
    for nx, ny in shapes:
        if ny > 1:
            W = wl.random_field_2d(gas, max(nx, ny), r, kmax=8, rms=1e-2)[:, :ny, :nx].copy()
            W[1] = 0.02 * r.normal(size=(ny, nx))
            W[2] = 0.02 * r.normal(size=(ny, nx))
        else:
            W = wl.multimode_1d(gas, nx, r, nmodes=16, kmax=64)
            W[1] = 0.02 * np.sin(2 * np.pi * np.arange(nx) / nx)
        s0 = ng.Solver(gas, nx, ny, W=W, precision=ng.NG_FP64)
        U = s0.conserved()
        s0.close()
        print(f"static step {case} {nx}x{ny}", flush=True)
        A, da = _step_static(ng, torch, gas, nx, ny, U, t=t, riemann=riemann, bc=bc,
                             scheme=scheme, source=source)
        B, db = _step_solver(ng, gas, nx, ny, U, t=t, riemann=riemann, bc=bc, scheme=scheme,
                             source=source)
        assert np.array_equal(A, B), (nx, ny, np.abs(A - B).max())
        assert da["t"] == db["t"] and da["dt_last"] == db["dt_last"] and da["steps"] == 1
        assert da["status"] == 0
        for q in range(5):
            assert da["total"][q] == pytest.approx(db["total"][q], rel=1e-13, abs=1e-15)


def test_static_step_refuses_what_it_cannot_do():
    """Another precision and a grid beyond the static scratch are refused
    before any device work, with a message."""
    import torch
    from paper_1805_03442_amd import ng
    assert torch.cuda.is_available()
    gas = dict(wl.BASE_GAS)
    dummy = torch.zeros(16, dtype=torch.float64, device="cuda")
    dummy2 = torch.zeros(16, dtype=torch.float64, device="cuda")
    rc = ng.lib().ng_step_static(C.byref(ng.make_gas(gas)), C.byref(ng.make_grid(64, 64)),
                                 C.byref(ng.make_numerics(precision=ng.NG_FP32)),
                                 C.c_void_p(dummy.data_ptr()), C.c_void_p(dummy2.data_ptr()), 0.0,
                                 0.0, C.c_void_p(ng.stream_handle()), None)
    assert rc == ng.NG_EINVAL and b"FP64" in ng.lib().ng_static_last_error()
    with pytest.raises(ng.NgError) as e:
        ng.step_static(gas, 16384, 16384, dummy, dummy2)
    assert e.value.code == ng.NG_ENOMEM and "static scratch" in str(e.value)
