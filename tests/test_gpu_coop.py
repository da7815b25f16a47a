"""GPU: the cooperative path (ng_set_coop).  One cooperative launch advances a
lone 1D solve through many steps of eq. (15), with a grid barrier per step
and the dt of eq. (16) chosen after each; its state, t and dt equal bit for
bit those of one launch per step on every kernel variant (closure recipes,
the general closures, HLL, walls and outflow), in every precision and in
both launch shapes (one wave per SIMD, and the largest workgroups the
kernel takes: 12 waves in FP32, 8 in FP64 and mixed; ragged tails).
A barrier wait that runs out of polls ends the launch with every kernel
exiting and leaves the solve at its last accepted step (NG_ESTALL).  Solves
with a forced source take the path too, MUSCL and CSPH-TVD."""
import sys

import numpy as np
import pytest

from paper_1805_03442_amd import workloads as wl

pytestmark = pytest.mark.gpu

W_, O_ = 1, 2


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ng():
    import torch
    assert torch.cuda.is_available()
    from paper_1805_03442_amd import ng as _ng
    _ng.lib()
    return _ng


def _state(gas, n, seed):
    """A moving multimode field: density modes plus a velocity wave."""
    W = wl.multimode_1d(gas, n, np.random.Generator(np.random.PCG64(seed)), nmodes=16,
                        kmax=min(64, n // 8), sigma=2e-3)
    x = (np.arange(n) + 0.5) / n
    W[1] = W[1] + 0.05 * np.sin(2 * np.pi * 3 * x)
    return W


# (name, cells, precision, riemann, x-end kinds, Q_T): the cells give 18 to
# 17477 segments, so one-wave-per-SIMD workgroups and the largest ones, one
# segment per wave and runs of several, with ragged last segments; 5 to 256
# workgroups, so one, two and four barrier slots per lane
CASES = [
    ("fp64_1024_hllc", 1024, "fp64", 0, (0, 0), 2.0),
    ("fp64_1003_hll_walls", 1003, "fp64", 1, (W_, O_), 2.0),
    ("fp64_131072_hllc", 1 << 17, "fp64", 0, (0, 0), 2.0),
    ("fp32_32768_recipe1", 32768, "fp32", 0, (0, 0), 2.0),
    ("fp32_100003_recipe2", 100003, "fp32", 0, (0, 0), 1.0),
    ("fp32_20000_general", 20000, "fp32", 0, (0, 0), 1.5),
    ("fp32_1048576_recipe1", 1 << 20, "fp32", 0, (0, 0), 2.0),
    ("fp32_5000_outflow_walls", 5000, "fp32", 0, (O_, W_), 2.0),
    ("mixed_70001_hll", 70001, "mixed", 1, (0, 0), 2.0),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_coop_equals_one_launch_per_step(ng, case):
    name, n, prec_name, riemann, ends, qt = case
    prec = {"fp64": ng.NG_FP64, "fp32": ng.NG_FP32, "mixed": ng.NG_MIXED}[prec_name]
    gas = dict(wl.BASE_GAS, Q_T=qt)
    W = _state(gas, n, 7 + n % 97)
    bc = (ends[0], ends[1], 0, 0)
    steps = 200
    say(f"coop case {name}: {steps} steps")
    a = ng.Solver(gas, n, 1, W=W, precision=prec, riemann=riemann, bc=bc)
    a.enable_timing(steps)
    a.step(steps)
    _, _, launches = a.kernel_time()
    assert launches == 1          # the whole run was one cooperative launch
    a.enable_timing(0)
    b = ng.Solver(gas, n, 1, W=W, precision=prec, riemann=riemann, bc=bc)
    b.set_coop(0)
    b.set_small_limit(0)
    b.step(steps)
    da, db = a.diagnostics(), b.diagnostics()
    assert da["status"] == 0 and db["status"] == 0
    assert da["steps"] == db["steps"] == steps
    for key in ("t", "dt_last", "dt_next", "smax", "rho_min", "p_min"):
        assert da[key] == db[key], key
    for q in (0, 3, 4):
        assert da["total"][q] == pytest.approx(db["total"][q], rel=1e-13)
    Ua, Ub = a.conserved(), b.conserved()
    assert np.array_equal(Ua, Ub)
    # a second call continues from the state the first one left
    a.run_to_time(da["t"] + 40 * da["dt_last"])
    b.run_to_time(db["t"] + 40 * db["dt_last"])
    assert a.diagnostics()["t"] == b.diagnostics()["t"]
    assert np.array_equal(a.conserved(), b.conserved())
    if prec == ng.NG_FP64 and n <= 2048:
        import oracle
        oracle.build()
        P = oracle.Problem(gas, n, 1, riemann=riemann, bc=bc)
        ref = P.run(P.prim_to_cons(W), steps)
        assert ref["status"] == 0
        assert np.array_equal(Ua[[0, 1, 3, 4]], ref["U"][[0, 1, 3, 4]])
        assert da["t"] == ref["t"]
    a.close()
    b.close()


def test_coop_lands_on_t_end(ng):
    """run_to_time on the cooperative path stops at t_end exactly, with the
    last step shortened as on the other paths."""
    gas = dict(wl.BASE_GAS, Q_T=2.0)
    W = _state(gas, 4096, 3)
    res = []
    for coop in (-1, 0):
        s = ng.Solver(gas, 4096, 1, W=W, precision=ng.NG_FP32)
        s.set_coop(coop)
        s.set_small_limit(0)
        taken = s.run_to_time(0.0123)
        d = s.diagnostics()
        assert d["t"] == 0.0123 and d["steps"] == taken
        res.append((s.conserved(), d["dt_last"]))
        s.close()
    assert np.array_equal(res[0][0], res[1][0]) and res[0][1] == res[1][1]


@pytest.mark.parametrize("n", [32768, 5000], ids=["137_workgroups", "21_workgroups"])
def test_coop_stall_ends_the_launch(ng, n):
    """With a spin limit of 0 polls every barrier wait gives up at once: the
    launch ends early with every workgroup leaving, the solve is stopped with
    NG_ESTALL at its last accepted step, whose state is bit for bit that of
    one launch per step, and later calls do not move it.  A new solve then
    runs normally (the device is unharmed).  Every workgroup waits for all
    the others' slots, so a step may or may not be accepted before the first
    wait gives up; 137 workgroups read four slots per lane, 21 one."""
    gas = dict(wl.BASE_GAS, Q_T=2.0)
    W = _state(gas, n, 5)
    s = ng.Solver(gas, n, 1, W=W, precision=ng.NG_FP32)
    s.set_coop(-1, 0)
    s.step(50)
    d = s.diagnostics()
    say(f"stalled launch: status {d['status']} after {d['steps']} steps")
    assert d["status"] == ng.NG_ESTALL
    k = d["steps"]
    assert 0 <= k < 50
    ref = ng.Solver(gas, n, 1, W=W, precision=ng.NG_FP32)
    ref.set_coop(0)
    ref.set_small_limit(0)
    if k:
        ref.step(k)
    assert np.array_equal(s.conserved(), ref.conserved())
    assert s.diagnostics()["t"] == ref.diagnostics()["t"]
    s.step(5)
    assert s.diagnostics()["steps"] == k
    with pytest.raises(ng.NgError) as err:
        s.run_to_time(1.0)
    assert err.value.code == ng.NG_ESTALL
    s.close()
    ref.close()
    t = ng.Solver(gas, n, 1, W=W, precision=ng.NG_FP32)
    t.step(20)
    assert t.diagnostics()["status"] == 0 and t.diagnostics()["steps"] == 20
    t.close()


def test_coop_is_not_taken_with_company(ng):
    """A batch of two solves keeps its own path (the cooperative path serves a
    lone 1D solve); a batch whose only solve is 1D takes it; results equal the
    per-step path."""
    gas = dict(wl.BASE_GAS, Q_T=2.0)
    n = 6000
    W = _state(gas, n, 9)
    b = ng.Batch(2, 1 << 26, precision=ng.NG_FP32)
    i = b.add(gas, n, 1, W, 10.0)
    b.run(30)
    alone = b.conserved(i)
    assert b.add(gas, n, 1, W, 10.0) is not None
    b.run(30)
    ref = ng.Solver(gas, n, 1, W=W, precision=ng.NG_FP32)
    ref.set_coop(0)
    ref.set_small_limit(0)
    ref.step(30)
    assert np.array_equal(alone, ref.conserved())
    ref.step(30)
    assert np.array_equal(b.conserved(i), ref.conserved())
    ref.close()
    b.close()


# forced sources (section 3) on the cooperative path: (name, cells, precision,
# scheme, riemann); the source's gas and wave are those of the paper's linear
# run, the cells give 14 to 100 segments and ragged last ones
SOURCE_CASES = [
    ("muscl_fp64_hllc_800", 800, "fp64", 0, 0),
    ("muscl_fp64_hll_3001", 3001, "fp64", 0, 1),
    ("muscl_fp32_hllc_6000", 6000, "fp32", 0, 0),
    ("muscl_mixed_hllc_2000", 2000, "mixed", 0, 0),
    ("csph_fp64_hll_1600", 1600, "fp64", 1, 1),
    ("csph_fp64_hll_5801", 5801, "fp64", 1, 1),
]


@pytest.mark.parametrize("case", SOURCE_CASES, ids=[c[0] for c in SOURCE_CASES])
def test_coop_with_a_forced_source_equals_one_launch_per_step(ng, case):
    """Every workgroup computes the source's ghosts for its own t each step
    (the wave at x = 0 reads them); the state, t and dt equal bit for bit
    those of one launch per step, whose ghosts come from the control block.
    After a cooperative call the control block holds the ghosts of its last
    step: per-step calls that follow continue bit for bit."""
    name, n, prec_name, scheme, riemann = case
    prec = {"fp64": ng.NG_FP64, "fp32": ng.NG_FP32, "mixed": ng.NG_MIXED}[prec_name]
    ws = wl.workload_forced_source("linear")
    gas, bc, src = ws["gas"], ws["bc"], ws["source"]
    W = wl.uniform_state(gas, n)
    steps = 300
    say(f"coop source case {name}: {steps} steps")

    def solver():
        return ng.Solver(gas, n, 1, W=W, precision=prec, riemann=riemann, bc=bc, source=src,
                         scheme=scheme)

    a = solver()
    a.enable_timing(steps)
    a.step(steps)
    assert a.kernel_time()[2] == 1    # one cooperative launch
    a.enable_timing(0)
    b = solver()
    b.set_coop(0)
    b.set_small_limit(0)
    b.step(steps)
    da, db = a.diagnostics(), b.diagnostics()
    assert da["status"] == 0 and db["status"] == 0 and da["steps"] == steps
    for key in ("t", "dt_last", "dt_next", "smax", "rho_min", "p_min"):
        assert da[key] == db[key], key
    assert np.array_equal(a.conserved(), b.conserved())
    # the wave has entered the domain
    assert np.abs(b.conserved()[0, :20] - gas["rho0"]).max() > 0.1 * src[0]
    # then one launch per step from the ghosts the cooperative call left
    a.set_coop(0)
    a.set_small_limit(0)
    a.step(40)
    b.step(40)
    assert a.diagnostics()["t"] == b.diagnostics()["t"]
    assert np.array_equal(a.conserved(), b.conserved())
    a.close()
    b.close()


def test_coop_random_configurations_equal_one_launch_per_step(ng):
    """30 seeded random configurations -- 5 to 2^20 cells; FP64, FP32, mixed;
    MUSCL with HLLC or HLL and CSPH-TVD; periodic, wall and outflow ends and
    section 3's forced source; closure exponents Q_T in {0, 1, 1.5, 2}; 1 to
    120 steps -- advance bit for bit alike on the cooperative path and with
    one launch per step (state, t, next dt, steps, status)."""
    r = np.random.Generator(np.random.PCG64(2026))
    src_gas = wl.workload_forced_source("linear")["gas"]
    for case in range(30):
        n = int(np.exp(r.uniform(np.log(5), np.log(1 << 20))))
        prec = [ng.NG_FP64, ng.NG_FP32, ng.NG_MIXED][int(r.integers(0, 3))]
        csph = prec == ng.NG_FP64 and r.random() < 0.3
        scheme = ng.NG_CSPH_TVD if csph else ng.NG_MUSCL
        riemann = ng.NG_HLL if csph else int(r.integers(0, 2))
        kind = int(r.integers(0, 3))
        qt = float(r.choice([0.0, 1.0, 1.5, 2.0]))
        gas, src = dict(wl.BASE_GAS, Q_T=qt), (0.0, 0.0)
        if kind == 0:
            bc = (0, 0, 0, 0)
        elif kind == 1:
            bc = (int(r.integers(1, 3)), int(r.integers(1, 3)), 0, 0)
        else:
            bc, src, gas = (3, 2, 0, 0), (1e-3, 0.1), src_gas
        if n >= 16:
            W = wl.multimode_1d(gas, n, r, nmodes=min(16, n // 8), kmax=min(64, n // 8),
                                sigma=1e-3)
        else:
            W = wl.uniform_state(gas, n)
        steps = int(r.integers(1, 120))
        say(f"random coop case {case}: n={n} prec={prec} scheme={scheme} riemann={riemann} "
            f"bc={bc} Q_T={qt} steps={steps}")
        res = []
        for coop in (True, False):
            s = ng.Solver(gas, n, 1, W=W, precision=prec, riemann=riemann, bc=bc, source=src,
                          scheme=scheme)
            if not coop:
                s.set_coop(0)
                s.set_small_limit(0)
            s.step(steps)
            d = s.diagnostics()
            res.append((s.conserved(), d["t"], d["dt_next"], d["steps"], d["status"]))
            s.close()
        assert np.array_equal(res[0][0], res[1][0]), case
        assert res[0][1:] == res[1][1:], (case, res[0][1:], res[1][1:])
