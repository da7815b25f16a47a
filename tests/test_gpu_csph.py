"""GPU: the CSPH-TVD step of section 2.3 (eqs. (9)-(14), 1D, FP64) through
the C ABI against the oracle (oracle/csph_oracle.c), bit for bit: state, t
and dt on periodic, wall and outflow ends, with sources and a body force,
on grids of 4 cells to a few thousand (one to many 58-cell wave segments,
ragged last segments), on every path a lone solve can take (one launch per
step, the persistent one-workgroup kernel, the cooperative kernel with a
grid barrier per step, captured graphs through run_to_time) and in several
launch shapes; at the size the benchmark times (2^22 cells) on two whole
steps; in a batch beside MUSCL solves; through the entry point that
allocates nothing; with a forced source (section 3).  The paper's own use
of the scheme as a cross-check: the blast waves of section 2.4 on 200 ...
1600 cells approach a fine MUSCL run (figure 2), and on section 3's
forced-source runs the two schemes agree better with every doubling.
"""
import sys

import numpy as np
import pytest

from paper_1805_03442_amd import workloads as wl

pytestmark = pytest.mark.gpu

W_, O_ = 1, 2
EULER = dict(wl.BASE_GAS, Cv=0.0, tau_rho=0.0, tau_T=0.0, Q0=0.0, Q_rho=0.0, Q_T=0.0,
             I0=0.0, I_rho=0.0, I_T=0.0, tau0=1.0)


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


@pytest.fixture(scope="module")
def oracle_mod():
    import oracle
    oracle.build()
    return oracle


def _moving_state(gas, n, seed):
    """Density, velocity and pressure fluctuations with flow towards and away
    from both ends."""
    r = np.random.Generator(np.random.PCG64(seed))
    W = wl.uniform_state(gas, n)
    x = (np.arange(n) + 0.5) / n
    W[0] *= 1.0 + 0.05 * r.standard_normal((1, n))
    W[1] = 0.2 * np.sin(2 * np.pi * x)[None, :] + 0.05 * r.standard_normal((1, n))
    W[3] *= 1.0 + 0.05 * r.standard_normal((1, n))
    return W


def _solver(ng, gas, n, U, bc, path, launch=None, source=(0.0, 0.0)):
    s = ng.Solver(gas, n, 1, U=U, precision=ng.NG_FP64, riemann=ng.NG_HLL, bc=bc,
                  scheme=ng.NG_CSPH_TVD, source=source)
    if path == "per_step":
        s.set_coop(0)
        s.set_small_limit(0)
    elif path == "small":
        s.set_coop(0)
        s.set_small_limit(1 << 30)
    if launch:
        s.set_launch(*launch)
    return s


# (name, cells, gas, x-end kinds, seed)
CASES = [
    ("periodic_1003_base", 1003, dict(wl.BASE_GAS, Q_T=2.0), (0, 0), 3),
    ("periodic_174_three_segments", 174, dict(wl.BASE_GAS, Q_T=2.0), (0, 0), 4),
    ("periodic_61", 61, dict(wl.BASE_GAS), (0, 0), 5),
    ("periodic_4", 4, dict(wl.BASE_GAS), (0, 0), 6),
    ("walls_1500", 1500, dict(wl.BASE_GAS, Q_T=2.0), (W_, W_), 7),
    ("outflow_wall_777", 777, dict(wl.BASE_GAS, Q_T=1.0), (O_, W_), 8),
    ("wall_outflow_59", 59, dict(wl.BASE_GAS), (W_, O_), 9),
    ("outflow_5", 5, dict(wl.BASE_GAS), (O_, O_), 10),
    ("euler_body_force_500", 500, dict(EULER, fx=3.0), (0, 0), 11),
    ("walls_body_force_300", 300, dict(wl.BASE_GAS, fx=-2.0), (W_, W_), 12),
]


@pytest.mark.parametrize("path", ["per_step", "small", "coop"])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_csph_bitwise_against_oracle(ng, oracle_mod, case, path):
    name, n, gas, ends, seed = case
    bc = (ends[0], ends[1], 0, 0)
    W = _moving_state(gas, n, seed)
    P = oracle_mod.CsphProblem(gas, n, bc=bc)
    U0 = P.prim_to_cons(W)
    steps = 120
    say(f"csph case {name} path {path}: {steps} steps")
    s = _solver(ng, gas, n, U0, bc, path)
    s.step(steps)
    d = s.diagnostics()
    U = s.conserved()
    s.close()
    ref = P.run(U0, steps)
    assert ref["status"] == 0 and d["status"] == 0
    assert d["steps"] == steps
    assert np.array_equal(U[[0, 1, 3, 4]], ref["U"][[0, 1, 3, 4]]), \
        np.abs(U - ref["U"]).max(axis=(1, 2))
    assert d["t"] == ref["t"] and d["dt_last"] == ref["dt_last"]
    # totals and the source budget: the same sums in another order
    h = 1.0 / n
    for q, c in ((0, 0), (1, 1), (3, 3), (4, 4)):
        assert d["total"][q] == pytest.approx(h * ref["U"][c].sum(), rel=1e-12, abs=1e-14)
    scale = h * np.abs(ref["U"][3]).sum()
    assert abs(d["src_budget"][0] - h * ref["budget"][0]) <= 1e-12 * scale
    assert abs(d["src_budget"][1] - h * ref["budget"][1]) <= 1e-12 * scale


@pytest.mark.parametrize("launch", [(1, 1), (2, 1), (3, 2), (8, 4)])
def test_csph_launch_shape_does_not_change_results(ng, oracle_mod, launch):
    """Segments per work item and waves per workgroup: each particle's
    arithmetic is that of its segment alone (two segments in a row also
    exercise the load of the next segment issued ahead)."""
    gas = dict(wl.BASE_GAS, Q_T=2.0)
    n = 2900
    W = _moving_state(gas, n, 21)
    bc = (W_, O_, 0, 0)
    P = oracle_mod.CsphProblem(gas, n, bc=bc)
    U0 = P.prim_to_cons(W)
    say(f"csph launch shape {launch}")
    s = _solver(ng, gas, n, U0, bc, "per_step", launch=launch)
    s.step(60)
    U = s.conserved()
    s.close()
    ref = P.run(U0, 60)
    assert np.array_equal(U[[0, 1, 3, 4]], ref["U"][[0, 1, 3, 4]])


@pytest.mark.parametrize("n", [200, 1600])
def test_csph_blast_waves_bitwise(ng, oracle_mod, n):
    """Section 2.4's blast waves between walls at the CSPH sizes of figure 2,
    run to t = 0.038 through captured graphs (run_to_time lands on t_end)."""
    bc = (W_, W_, 0, 0)
    P = oracle_mod.CsphProblem(EULER, n, bc=bc)
    U0 = P.prim_to_cons(wl.blast_waves_1d(n))
    say(f"csph blast waves n={n}")
    for path in ("per_step", "small", "coop"):
        s = _solver(ng, EULER, n, U0, bc, path)
        taken = s.run_to_time(0.038)
        d = s.diagnostics()
        U = s.conserved()
        s.close()
        ref = P.run(U0, 10 ** 7, t_end=0.038)
        assert ref["status"] == 0 and d["status"] == 0
        assert d["t"] == 0.038 and taken == ref["steps"]
        assert np.array_equal(U[[0, 1, 3, 4]], ref["U"][[0, 1, 3, 4]])


def test_csph_full_size_two_steps(ng, oracle_mod):
    """The benchmark's grid (2^22 cells, periodic, 64 random modes plus a
    velocity wave) in its launch configuration: two whole steps equal the
    oracle's everywhere."""
    n = 1 << 22
    gas = dict(wl.BASE_GAS, Q_T=2.0)
    W = wl.workload_csph_1d(n)["W"]
    P = oracle_mod.CsphProblem(gas, n)
    U0 = P.prim_to_cons(W)
    say("csph full size: 2 steps on the GPU")
    s = ng.Solver(gas, n, 1, U=U0, precision=ng.NG_FP64, riemann=ng.NG_HLL,
                  scheme=ng.NG_CSPH_TVD)
    s.step(2)
    d = s.diagnostics()
    U = s.conserved()
    s.close()
    say("csph full size: 2 oracle steps")
    ref = P.run(U0, 2)
    assert d["status"] == 0 and ref["status"] == 0
    assert np.array_equal(U[[0, 1, 3, 4]], ref["U"][[0, 1, 3, 4]])
    assert d["t"] == ref["t"]


@pytest.mark.parametrize("n", [3000, 1 << 17, 100003])
def test_csph_cooperative_equals_one_launch_per_step(ng, n):
    """A lone CSPH solve runs as one cooperative launch (one wave per SIMD
    for a few segments, 8-wave workgroups with runs of segments beyond);
    state, t and dt equal one launch per step bit for bit, and a second call
    continues from the first."""
    gas = dict(wl.BASE_GAS, Q_T=2.0)
    W = _moving_state(gas, n, 31 + n % 7)
    bc = (W_, O_, 0, 0) if n == 100003 else (0, 0, 0, 0)
    say(f"csph cooperative n={n}")
    a = ng.Solver(gas, n, 1, W=W, precision=ng.NG_FP64, riemann=ng.NG_HLL, bc=bc,
                  scheme=ng.NG_CSPH_TVD)
    a.enable_timing(150)
    a.step(150)
    assert a.kernel_time()[2] == 1
    a.enable_timing(0)
    b = ng.Solver(gas, n, 1, W=W, precision=ng.NG_FP64, riemann=ng.NG_HLL, bc=bc,
                  scheme=ng.NG_CSPH_TVD)
    b.set_coop(0)
    b.set_small_limit(0)
    b.step(150)
    da, db = a.diagnostics(), b.diagnostics()
    assert da["status"] == 0 and db["status"] == 0 and da["steps"] == db["steps"] == 150
    for key in ("t", "dt_last", "dt_next", "smax", "rho_min", "p_min"):
        assert da[key] == db[key], key
    assert np.array_equal(a.conserved(), b.conserved())
    a.run_to_time(da["t"] + 30 * da["dt_last"])
    b.run_to_time(db["t"] + 30 * db["dt_last"])
    assert a.diagnostics()["t"] == b.diagnostics()["t"]
    assert np.array_equal(a.conserved(), b.conserved())
    a.close()
    b.close()


def test_csph_shares_a_batch_with_muscl(ng, oracle_mod):
    """In an FP64 batch beside MUSCL solves every member equals its own lone
    run bit for bit (the batch's 1D launch takes the general kernel, which
    branches per solve)."""
    gas = dict(wl.BASE_GAS, Q_T=2.0)
    n = 3000
    W = _moving_state(gas, n, 31)
    P = oracle_mod.CsphProblem(gas, n)
    s = _solver(ng, gas, n, P.prim_to_cons(W), (0, 0, 0, 0), "per_step")
    s.step(25)
    lone_csph = s.conserved()
    s.close()
    m = ng.Solver(gas, n, 1, W=W, precision=ng.NG_FP64, riemann=ng.NG_HLL)
    m.set_coop(0)
    m.step(25)
    lone_muscl = m.conserved()
    m.close()
    say("csph in a batch with MUSCL solves")
    b = ng.Batch(4, 1 << 27, precision=ng.NG_FP64)
    i = b.add(gas, n, 1, W, 10.0, riemann=ng.NG_HLL, scheme=ng.NG_CSPH_TVD)
    j = b.add(gas, n, 1, W, 10.0, riemann=ng.NG_HLL)
    k = b.add(gas, 700, 1, W[:, :, :700], 10.0, riemann=ng.NG_HLL, scheme=ng.NG_CSPH_TVD)
    b.run(25)
    assert np.array_equal(b.conserved(i), lone_csph)
    assert np.array_equal(b.conserved(j), lone_muscl)
    P = oracle_mod.CsphProblem(gas, 700)
    ref = P.run(P.prim_to_cons(W[:, :, :700]), 25)
    assert np.array_equal(b.conserved(k)[[0, 1, 3, 4]], ref["U"][[0, 1, 3, 4]])
    b.close()


def _sink_case():
    """A strong energy sink independent of temperature (I0 = 20, I_T = 0)
    drives the pressure negative after some tens of steps."""
    gas = dict(wl.BASE_GAS, I0=20.0, I_T=0.0)
    return gas, wl.acoustic_mode_1d(gas, 300, 3, 1e-2), 300


@pytest.mark.parametrize("path", ["per_step", "small", "coop"])
def test_csph_rejected_step_keeps_last_good_state(ng, oracle_mod, path):
    """The step that produces p <= 0 is rejected at the oracle's step
    (NG_EPHYS); the solve keeps the oracle's last good state bit for bit and
    does not move on."""
    gas, W, n = _sink_case()
    P = oracle_mod.CsphProblem(gas, n)
    U0 = P.prim_to_cons(W)
    ref = P.run(U0, 2000)
    assert ref["status"] != 0
    say(f"csph sink case {path}: oracle stops after {ref['steps']} steps")
    s = _solver(ng, gas, n, U0, (0, 0, 0, 0), path)
    with pytest.raises(ng.NgError) as err:
        s.run_to_time(10.0, 2000)
    assert err.value.code == ng.NG_EPHYS
    d = s.diagnostics()
    assert d["status"] != 0 and d["steps"] == ref["steps"]
    assert d["t"] == ref["t"]
    assert np.array_equal(s.conserved()[[0, 1, 3, 4]], ref["U"][[0, 1, 3, 4]])
    s.step(5)
    assert s.diagnostics()["steps"] == ref["steps"]
    s.close()


def test_csph_blast_waves_approach_the_fine_muscl_run(ng):
    """Figure 2's comparison: the CSPH-TVD density at t = 0.038 on 200, 400,
    800 and 1600 cells against a 64000-cell MUSCL run averaged onto each grid
    (the paper's reference is a 10^5-cell run): the L1 difference falls with
    every doubling and by at least 2.5 from 200 to 1600 cells; the density
    peak of the finest CSPH run lies near x = 0.78 and within 10 % of the
    reference's."""
    bc = (W_, W_, 0, 0)

    def run(n, scheme, riemann):
        s = ng.Solver(EULER, n, 1, W=wl.blast_waves_1d(n), precision=ng.NG_FP64,
                      riemann=riemann, bc=bc, scheme=scheme)
        s.run_to_time(0.038, 10 ** 7)
        d = s.diagnostics()
        rho = s.conserved()[0, 0]
        s.close()
        assert d["status"] == 0 and d["t"] == 0.038
        return rho, d["steps"]

    nf = 64000
    rf, steps = run(nf, ng.NG_MUSCL, ng.NG_HLLC)
    say(f"fine MUSCL run n={nf}: {steps} steps")
    errs = []
    for n in (200, 400, 800, 1600):
        rho, steps = run(n, ng.NG_CSPH_TVD, ng.NG_HLL)
        avg = rf.reshape(n, nf // n).mean(axis=1)
        errs.append(float(np.mean(np.abs(rho - avg))))
        say(f"csph n={n}: {steps} steps, L1 difference {errs[-1]:.4f}")
    assert all(b < a for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < errs[0] / 2.5, errs
    jf = int(np.argmax(rf))
    assert abs((np.argmax(rho) + 0.5) / 1600 - (jf + 0.5) / nf) < 0.01
    assert abs(rho.max() - rf.max()) < 0.1 * rf.max()


@pytest.mark.parametrize("path", ["per_step", "small", "coop"])
@pytest.mark.parametrize("stage", ["linear", "nonlinear"])
def test_csph_forced_source_against_oracle(ng, oracle_mod, stage, path):
    """Section 3's forced source with the CSPH-TVD step: the three ghost
    particles before x = 0 carry the source's wave at each step's start time.
    400 steps of both runs' media; FP64 within 1e-12 of the oracle per
    component (the device sine of the source may differ from libm's in the
    last bit, so not bit for bit), t within 1e-13."""
    ws = wl.workload_forced_source(stage)
    n, steps = ws["nx"], 400
    P = oracle_mod.CsphProblem(ws["gas"], n, bc=ws["bc"], source=ws["source"])
    U0 = P.prim_to_cons(ws["W"])
    ref = P.run(U0, steps)
    assert ref["status"] == 0
    say(f"csph forced source {stage} {path}")
    s = _solver(ng, ws["gas"], n, U0, ws["bc"], path, source=ws["source"])
    s.step(steps)
    d = s.diagnostics()
    U = s.conserved()
    s.close()
    assert d["status"] == 0 and d["steps"] == steps
    for c in (0, 1, 3, 4):
        den = np.max(np.abs(ref["U"][c]))
        assert np.max(np.abs(U[c] - ref["U"][c])) <= 1e-12 * den, c
    assert d["t"] == pytest.approx(ref["t"], rel=1e-13)
    # the wave has entered the domain
    dr = np.abs(ref["U"][0, 0] - ws["gas"]["rho0"])
    assert dr[: n // 20].max() > 0.1 * ws["source"][0]


@pytest.mark.parametrize("stage", ["linear", "nonlinear"])
def test_csph_cross_checks_muscl_on_the_forced_source_runs(ng, stage):
    """The paper's use of its second scheme: section 3's two forced-source
    runs to t = 0.8 (the linear stage and the shock train) with CSPH-TVD and
    with MUSCL on 800, 1600 and 3200 cells.  The velocity fields agree
    better with every doubling (relative L1 difference halving: CSPH-TVD is
    first order for sound, reading 22) and within 6 % on 3200 cells."""
    ws = wl.workload_forced_source(stage)
    diffs = []
    for n in (800, 1600, 3200):
        u = {}
        for name, scheme, riemann in (("csph", ng.NG_CSPH_TVD, ng.NG_HLL),
                                      ("muscl", ng.NG_MUSCL, ng.NG_HLLC)):
            s = ng.Solver(ws["gas"], n, 1, W=wl.uniform_state(ws["gas"], n),
                          precision=ng.NG_FP64, riemann=riemann, bc=ws["bc"],
                          source=ws["source"], scheme=scheme)
            s.run_to_time(ws["t_end"])
            d = s.diagnostics()
            U = s.conserved()
            s.close()
            assert d["status"] == 0 and d["t"] == ws["t_end"]
            u[name] = U[1, 0] / U[0, 0]
        diffs.append(float(np.abs(u["csph"] - u["muscl"]).sum() / np.abs(u["muscl"]).sum()))
        say(f"forced source {stage} n={n}: CSPH against MUSCL {diffs[-1]:.4f}")
    assert all(a / b > 1.8 for a, b in zip(diffs, diffs[1:])), diffs
    assert diffs[-1] < 0.06, diffs
