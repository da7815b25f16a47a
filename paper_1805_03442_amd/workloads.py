"""Seeded synthetic inputs: gas parameters and FP64 primitive initial states.

This module holds only input recipes (random draws, sinusoids, spectra).  It
contains none of the scheme's arithmetic, so the oracle and the HIP path can
both be fed from it.  Every array is primitive and FP64, laid out as
``W[5, ny, nx]`` = (rho, u, v, p, E_nu) with cell (j, k) centred at
``((j + 1/2) h, (k + 1/2) h)``; a 1D state has ``ny == 1`` and ``v == 0``.

The paper runs no public dataset; all of its test problems are defined by
formulas.  The five workloads below follow the parameter sets of the solver
specification (1D acoustic mode, 1D multi-mode, 2D random field, a batch of
uneven 1D instances and a served request stream); units are those of the
paper's section 2.3 (rho_0, p_0, sqrt(p_0/rho_0)), so rho_0 = p_0 = R = T_0 = 1.
"""
from __future__ import annotations

import math

import numpy as np

SEED_BASE = 1805034420

# Base gas of the workloads: eqs. (5)-(7) with the closures (6).
BASE_GAS = dict(gamma=1.4, R=1.0, Cv=1.0, rho0=1.0, T0=1.0,
                tau0=0.05, tau_rho=-1.0, tau_T=-1.0,
                Q0=0.1, Q_rho=0.5, Q_T=1.0,
                I0=0.1, I_rho=1.0, I_T=2.0,
                fx=0.0, fy=0.0)
CFL = 0.4


def rng(config_index: int) -> np.random.Generator:
    """PCG64 stream of one workload (config_index counts from 1)."""
    return np.random.Generator(np.random.PCG64(SEED_BASE + int(config_index)))


def background(gas: dict) -> dict:
    """Uniform background: rho0, u = v = 0, p = R rho0 T0 and the vibrational
    energy at which relaxation balances the pump in eq. (4):
    E_nu0 = rho0 Cv T0 + rho0 tau0 Q0 (steady when Q0 = I0 in eq. (3))."""
    rho0, T0 = gas["rho0"], gas["T0"]
    p0 = gas["R"] * rho0 * T0
    ev0 = rho0 * gas["Cv"] * T0 + rho0 * gas["tau0"] * gas["Q0"]
    return dict(rho=rho0, p=p0, ev=ev0)


def uniform_state(gas: dict, nx: int, ny: int = 1) -> np.ndarray:
    b = background(gas)
    W = np.zeros((5, ny, nx))
    W[0] = b["rho"]
    W[3] = b["p"]
    W[4] = b["ev"]
    return W


def cell_centres(n: int, L: float = 1.0) -> np.ndarray:
    h = L / n
    return (np.arange(n) + 0.5) * h


def _apply_density_perturbation(gas: dict, W: np.ndarray, drho: np.ndarray,
                                du: np.ndarray | None = None) -> np.ndarray:
    """Isentropic (frozen) companion of a density perturbation: dp = c^2 drho
    with c^2 = gamma p0 / rho0, specific vibrational energy E_nu/rho unchanged."""
    b = background(gas)
    c2 = gas["gamma"] * b["p"] / b["rho"]
    W[0] = b["rho"] + drho
    W[3] = b["p"] + c2 * drho
    W[4] = b["ev"] * (W[0] / b["rho"])
    if du is not None:
        W[1] = du
    return W


def acoustic_mode_1d(gas: dict, n: int, mode: int, amp: float,
                     mode_vector=None) -> np.ndarray:
    """One right-going sound wave of wavenumber k = 2 pi mode on [0, 1).

    By default the frozen isentropic wave: drho = amp sin(k x), u = c drho/rho0,
    dp = c^2 drho, E_nu/rho unchanged.  ``mode_vector`` may instead give the
    complex amplitudes (rho, u, p, E_nu) of any linear mode, normalised so that
    the density amplitude is ``amp``: field = Re(a exp(i k x)) with a the vector
    times -i (so that the density is amp sin(k x) for a real density entry)."""
    x = cell_centres(n)
    W = uniform_state(gas, n)
    k = 2.0 * math.pi * mode
    if mode_vector is None:
        b = background(gas)
        c = math.sqrt(gas["gamma"] * b["p"] / b["rho"])
        drho = amp * np.sin(k * x)
        _apply_density_perturbation(gas, W.reshape(5, n), drho, c * drho / b["rho"])
        return W
    v = np.asarray(mode_vector, dtype=np.complex128)
    v = v / v[0] * amp
    phase = np.exp(1j * k * x) * (-1j)
    b = background(gas)
    W[0, 0] = b["rho"] + np.real(v[0] * phase)
    W[1, 0] = np.real(v[1] * phase)
    W[3, 0] = b["p"] + np.real(v[2] * phase)
    W[4, 0] = b["ev"] + np.real(v[3] * phase)
    return W


def multimode_1d(gas: dict, n: int, r: np.random.Generator, nmodes: int = 64,
                 kmax: int = 256, sigma: float = 1e-4) -> np.ndarray:
    """Sum of ``nmodes`` distinct integer modes drawn from 1..kmax with phases
    U[0, 2 pi) and amplitudes N(0, sigma), on the density; isentropic companion.

    The sum of sines a_m sin(2 pi m x_j + phi_m), x_j = (j + 1/2)/n, is
    synthesised by one inverse real FFT: it is Re sum_m X_m exp(2 pi i m j / n)
    with X_m = -i a_m exp(i (phi_m + pi m / n)) (modes below n/2)."""
    modes = np.sort(r.choice(np.arange(1, kmax + 1), size=nmodes, replace=False))
    phases = r.uniform(0.0, 2.0 * math.pi, size=nmodes)
    amps = r.normal(0.0, sigma, size=nmodes)
    if 2 * int(modes.max()) >= n:
        raise ValueError("modes must lie below n/2")
    X = np.zeros(n // 2 + 1, dtype=np.complex128)
    X[modes] = -1j * amps * np.exp(1j * (phases + math.pi * modes / n)) * (n / 2.0)
    drho = np.fft.irfft(X, n)
    W = uniform_state(gas, n)
    _apply_density_perturbation(gas, W.reshape(5, n), drho)
    return W


def random_field_2d(gas: dict, n: int, r: np.random.Generator, kmax: int = 64,
                    rms: float = 1e-3, slope: float = -2.0) -> np.ndarray:
    """Isotropic Gaussian random density field on an n x n periodic grid:
    integer wave-vectors with 1 <= |k| <= kmax, complex normal coefficients of
    variance |k|^slope, Hermitian by taking the real part of the inverse FFT,
    rescaled to the requested rms; isentropic pressure, v = 0."""
    kx = np.fft.fftfreq(n, d=1.0 / n)
    KX, KY = np.meshgrid(kx, kx, indexing="xy")
    kk = np.sqrt(KX * KX + KY * KY)
    mask = (kk >= 1.0) & (kk <= kmax)
    amp = np.zeros((n, n))
    amp[mask] = kk[mask] ** (slope / 2.0)
    coef = (r.normal(size=(n, n)) + 1j * r.normal(size=(n, n))) * amp
    field = np.real(np.fft.ifft2(coef))
    field *= rms / np.sqrt(np.mean(field * field))
    W = np.zeros((5, n, n))
    b = background(gas)
    W[0] = b["rho"]
    W[3] = b["p"]
    W[4] = b["ev"]
    _apply_density_perturbation(gas, W.reshape(5, n * n), field.reshape(-1))
    return W


def riemann_tophat(gas: dict, n: int, left: tuple, right: tuple) -> np.ndarray:
    """Two Riemann problems on a periodic [0, 1): state ``left`` (rho, u, p, E_nu)
    on [1/4, 3/4) and ``right`` elsewhere, so that the interface at x = 3/4 is a
    left/right problem and the one at 1/4 its mirror image."""
    x = cell_centres(n)
    inner = (x >= 0.25) & (x < 0.75)
    W = np.zeros((5, 1, n))
    for c, (a, b) in zip((0, 1, 3, 4), zip(left, right)):
        W[c, 0] = np.where(inner, a, b)
    return W


def blast_waves_1d(n: int) -> np.ndarray:
    """Two interacting blast waves of section 2.4 (rho = 1, u = 0; p = 1000 on
    [0, 0.1), 0.01 on [0.1, 0.9], 100 on (0.9, 1]), no vibrational energy."""
    x = cell_centres(n)
    W = np.zeros((5, 1, n))
    W[0, 0] = 1.0
    W[3, 0] = np.where(x < 0.1, 1000.0, np.where(x <= 0.9, 0.01, 100.0))
    return W


def results_gas(S: float, tau0: float = 1.0) -> dict:
    """Gas of the runs of section 3: gamma = 1.4, C_k = Cv / R = 0.1, tau_rho
    = -1, tau_T = -1.5, Q and I exponents 0, rho0 = p0 = 1 and tau0 = 1 (the
    units), and the degree of non-equilibrium S = tau0 Q0 / (R T0) through
    Q0 = I0 = S R T0 / tau0 (pump and sink balance on the background)."""
    q = S / tau0
    return dict(gamma=1.4, R=1.0, Cv=0.1, rho0=1.0, T0=1.0, tau0=tau0, tau_rho=-1.0,
                tau_T=-1.5, Q0=q, Q_rho=0.0, Q_T=0.0, I0=q, I_rho=0.0, I_T=0.0,
                fx=0.0, fy=0.0)


# ------------------------------------------------------------------ workloads

def workload_1d_acoustic():
    """1D periodic, 1024 cells, FP64, one acoustic mode k = 2 pi * 4, amplitude
    1e-3, base gas, 2000 steps."""
    gas = dict(BASE_GAS)
    W = acoustic_mode_1d(gas, 1024, 4, 1e-3)
    return dict(name="1d_acoustic_n1024", gas=gas, W=W, nx=1024, ny=1, steps=2000,
                precision="fp64")


def workload_1d_multimode(n: int = 1 << 20):
    """1D periodic, 2^20 cells, Q_T = 2, 64 random modes in 1..256 with N(0, 1e-4)
    amplitudes, 20000 steps."""
    gas = dict(BASE_GAS, Q_T=2.0)
    W = multimode_1d(gas, n, rng(2))
    return dict(name=f"1d_multimode_n{n}", gas=gas, W=W, nx=n, ny=1, steps=20000,
                precision="fp32")


def workload_csph_1d(n: int = 1 << 22):
    """1D periodic, 2^22 cells, Q_T = 2: 64 random density modes in 1..256
    with N(0, 1e-3) amplitudes (isentropic pressure) on a velocity wave
    0.05 sin(2 pi 3 x), so that the particles of the CSPH-TVD step move;
    FP64, HLL."""
    gas = dict(BASE_GAS, Q_T=2.0)
    W = multimode_1d(gas, n, rng(5), sigma=1e-3)
    W[1, 0] = 0.05 * np.sin(2.0 * math.pi * 3.0 * cell_centres(n))
    return dict(name=f"1d_csph_multimode_n{n}", gas=gas, W=W, nx=n, ny=1, steps=2000,
                precision="fp64")


def workload_2d_random(n: int = 4096):
    """2D periodic n x n (4096^2), Q_T = 2, isotropic k^-2 density field with
    |k| <= 64 and rms 1e-3, 5000 steps."""
    gas = dict(BASE_GAS, Q_T=2.0)
    W = random_field_2d(gas, n, rng(3))
    return dict(name=f"2d_random_{n}x{n}", gas=gas, W=W, nx=n, ny=n, steps=5000,
                precision="fp32")


def workload_forced_source(stage: str = "nonlinear"):
    """The 1D runs of section 3: a source at x = 0 emits sound of wavelength
    0.1 into the uniform background (free outflow at x = 1), t = 0.8.  Linear
    stage: S = 0.5, N = 800; nonlinear stage: S = 1, N = 1600.  The paper
    states no source amplitude; the readings are 1e-3 (linear) and 3e-2
    (nonlinear: a simple wave of that amplitude steepens into shocks within
    about 0.4 of travel, so the domain holds a shock train by t = 0.8)."""
    if stage == "linear":
        S, n, amp = 0.5, 800, 1e-3
    else:
        S, n, amp = 1.0, 1600, 3e-2
    gas = results_gas(S)
    return dict(name=f"forced_source_{stage}_S{S:g}_n{n}", gas=gas, W=uniform_state(gas, n),
                nx=n, ny=1, bc=(3, 2, 0, 0), source=(amp, 0.1), t_end=0.8)


def sector_active(n: int, L: float, x0: float, y0: float, tan: float) -> np.ndarray:
    """Cells (ny, nx) of an n x n grid of side L whose centre lies in the wedge
    x >= x0, |y - y0| <= (x - x0) tan (the active medium of the sector run)."""
    h = L / n
    x = (np.arange(n) + 0.5) * h
    y = (np.arange(n) + 0.5) * h
    dx = x[None, :] - x0
    return (dx >= 0.0) & (np.abs(y[:, None] - y0) <= dx * tan)


def workload_sector_2d(n: int = 600, S: float = 1.0, tau0: float = 1.0, amp: float = 1e-2,
                       L: float = 1.2, t_end: float = 1.0):
    """The 2D run of section 3: the active medium fills a sector of opening
    angle 30 degrees whose apex is the source, the rest of the gas is passive
    (no pump or sink); a wall G1 and free flow G2-G4.  The geometry is shown
    only in a figure; the readings: square domain of side L = 1.2 (so the
    wave meets G1 at t ~ 1, as the paper states), source on the x-low edge at
    y = L/2 over one wavelength (|y - L/2| <= 0.05), the rest of that edge and
    both y edges free outflow (G2-G4), the x-high edge a wall (G1), the sector
    symmetric about y = L/2 with its apex at the source.  The initial state is
    the steady background of each medium (E_nu carries rho tau0 Q0 only in
    the active part)."""
    gas = results_gas(S, tau0)
    lam = 0.1
    x0, y0, tan = 0.0, 0.5 * L, math.tan(math.radians(15.0))
    act = sector_active(n, L, x0, y0, tan)
    b = background(gas)
    W = np.zeros((5, n, n))
    W[0] = b["rho"]
    W[3] = b["p"]
    W[4] = gas["rho0"] * gas["Cv"] * gas["T0"] + np.where(act, gas["rho0"] * gas["tau0"] * gas["Q0"], 0.0)
    return dict(name=f"sector_2d_S{S:g}_n{n}", gas=gas, W=W, nx=n, ny=n, h=L / n,
                bc=(3, 1, 2, 2), source=(amp, lam, 0.5 * L, 0.5 * lam),
                wedge=(x0, y0, tan), t_end=t_end, active=act)


def batch_1d_instances(count: int = 512, nmin_log2: float = 10.0, nmax_log2: float = 16.0,
                       steps: int = 10000):
    """Batch of uneven 1D periodic instances: n log-uniform in [2^10, 2^16],
    tau0 ~ U[0.005, 0.5], Q_T ~ U[0, 3], one acoustic mode m ~ U{1..16} of
    amplitude 1e-3.  Returns a list of instance dicts (gas, W, nx, mode)."""
    r = rng(4)
    out = []
    for i in range(count):
        n = int(round(2.0 ** r.uniform(nmin_log2, nmax_log2)))
        gas = dict(BASE_GAS, tau0=float(r.uniform(0.005, 0.5)), Q_T=float(r.uniform(0.0, 3.0)))
        m = int(r.integers(1, 17))
        W = acoustic_mode_1d(gas, n, m, 1e-3)
        out.append(dict(gas=gas, W=W, nx=n, ny=1, mode=m, steps=steps))
    return out


def serve_trace(count: int = 2000, rate: float = 200.0, seed_offset: int = 0,
                log2_1d=(12.0, 20.0), side_2d=(256.0, 2048.0), t_end=(0.1, 2.0),
                frac_1d: float = 0.5):
    """Served request stream: Poisson arrivals at ``rate`` per second; half 1D
    (n log-uniform 2^12..2^20), half 2D (side log-uniform 256..2048); base gas
    with Q_T = 2 and per-request tau0 ~ U[0.005, 0.5], Q_T ~ U[0, 3];
    t_end ~ U[0.1, 2].  The initial data are drawn when a request is
    materialised (``request_state``), from the request's own seed."""
    r = rng(5 + seed_offset)
    t = 0.0
    reqs = []
    for i in range(count):
        t += r.exponential(1.0 / rate)
        is1d = r.uniform() < frac_1d
        if is1d:
            nx = int(round(2.0 ** r.uniform(*log2_1d)))
            ny = 1
        else:
            nx = int(round(2.0 ** r.uniform(math.log2(side_2d[0]), math.log2(side_2d[1]))))
            ny = nx
        gas = dict(BASE_GAS, Q_T=float(r.uniform(0.0, 3.0)), tau0=float(r.uniform(0.005, 0.5)))
        reqs.append(dict(id=i, arrival=t, nx=nx, ny=ny, gas=gas,
                         t_end=float(r.uniform(*t_end)),
                         seed=int(r.integers(0, 2**31 - 1))))
    return reqs


def modes_2d(gas: dict, n: int, r: np.random.Generator, nmodes: int = 8, kmax: int = 16,
             rms: float = 1e-3) -> np.ndarray:
    """A few random plane waves on an n x n periodic grid: integer wave-vectors
    with components in [-kmax, kmax], random phases, Gaussian amplitudes,
    rescaled to the requested rms; isentropic pressure, v = 0.  Built as one
    (n x 2m) by (2m x n) product of separable factors, for request streams."""
    x = cell_centres(n)
    Y = np.zeros((2 * nmodes, n))
    X = np.zeros((2 * nmodes, n))
    for m in range(nmodes):
        kx, ky = r.integers(-kmax, kmax + 1, size=2)
        if kx == 0 and ky == 0:
            kx = 1
        ph = r.uniform(0.0, 2.0 * math.pi)
        a = r.normal()
        # sin(p + q) = sin p cos q + cos p sin q, p along x, q along y
        px = 2.0 * math.pi * kx * x + ph
        qy = 2.0 * math.pi * ky * x
        Y[2 * m] = a * np.cos(qy)
        X[2 * m] = np.sin(px)
        Y[2 * m + 1] = a * np.sin(qy)
        X[2 * m + 1] = np.cos(px)
    field = Y.T @ X
    field *= rms / max(np.sqrt(np.mean(field * field)), 1e-300)
    W = np.empty((5, n, n))
    b = background(gas)
    W[1] = 0.0
    W[2] = 0.0
    _apply_density_perturbation(gas, W.reshape(5, n * n), field.reshape(-1))
    return W


def request_state(req: dict) -> np.ndarray:
    """Initial state of one served request, drawn from the request's own seed:
    16 random modes in 1D, 8 random plane waves in 2D (wavenumbers small enough
    for the request's grid)."""
    r = np.random.Generator(np.random.PCG64(req["seed"]))
    nx, ny = req["nx"], req["ny"]
    if ny == 1:
        return multimode_1d(req["gas"], nx, r, nmodes=16, kmax=min(256, nx // 8))
    return modes_2d(req["gas"], nx, r, nmodes=8, kmax=max(1, min(16, nx // 16)))
