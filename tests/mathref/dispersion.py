"""Linear theory of section 2.2: small plane waves on the uniform steady state.

A pin for the oracle, independent of it.  Two routes to the same roots:

* ``matrix(gas, k)`` linearises eqs. (1)-(7) in 1D about the steady background
  (u = 0, p0 = R rho0 T0, Q0 = I0, E_nu0 - E_nue0 = rho0 tau0 Q0) with the
  closures (6) and E_nue = rho Cv T, in the unknowns (rho', u', p', E_nu').  A
  perturbation exp(-i omega t + i k x) obeys -i omega X = M X, so omega = i
  * eig(M) and the temporal growth rate is Im omega = Re eig(M).
* ``paper_residual(gas, omega, k)`` is the dispersion equation (8) as printed,
  with C_k = dE_nue/(R dT) per unit mass (= Cv/R here) and S = tau0 Q0/(R T0).
  One factor of the left-hand side is garbled in the source text ("(1 - i
  delta) gamma_1/(delta R)"); it is read as (1 - i delta) gamma_1/(omega R T0),
  the form that matches the right-hand side's factor and makes every term
  dimensionless.

The eigenvalues of ``matrix`` are checked to be roots of (8) in the tests.
"""
from __future__ import annotations

import numpy as np


def background(gas):
    rho0, T0 = gas["rho0"], gas["T0"]
    p0 = gas["R"] * rho0 * T0
    ev0 = rho0 * gas["Cv"] * T0 + rho0 * gas["tau0"] * gas["Q0"]
    return rho0, p0, T0, ev0


def matrix(gas, k):
    """M(k) with -i omega X = M X for X = (rho', u', p', E_nu')."""
    g = gas
    rho0, p0, T0, ev0 = background(g)
    gam, gm1, R, Cv = g["gamma"], g["gamma"] - 1.0, g["R"], g["Cv"]
    tau0, Q0, I0 = g["tau0"], g["Q0"], g["I0"]
    ik = 1j * k
    # d(T'/T0)/dX and d(rho'/rho0)/dX as row vectors over (rho', u', p', E_nu')
    dr = np.array([1.0 / rho0, 0.0, 0.0, 0.0])
    dT = np.array([-1.0 / rho0, 0.0, 1.0 / p0, 0.0])
    dtau_over_tau = g["tau_rho"] * dr + g["tau_T"] * dT          # tau'/tau0
    dQ = Q0 * (g["Q_rho"] * dr + g["Q_T"] * dT)                   # Q'
    dI = I0 * (g["I_rho"] * dr + g["I_T"] * dT)                   # I'
    dEe = np.array([0.0, 0.0, Cv / R, 0.0])                       # E_nue' = Cv p'/R
    dEv = np.array([0.0, 0.0, 0.0, 1.0])
    drho = np.array([1.0, 0.0, 0.0, 0.0])
    M = np.zeros((4, 4), dtype=np.complex128)
    # continuity: rho_t = -rho0 u_x
    M[0, 1] = -ik * rho0
    # momentum: u_t = -p_x / rho0
    M[1, 2] = -ik / rho0
    # pressure: p_t = -gamma p0 u_x + (gamma-1) [(E_nu - E_nue)/tau - rho I]
    relax = (dEv - dEe) / tau0 - (ev0 - rho0 * Cv * T0) * dtau_over_tau / tau0
    M[2, :] += gm1 * (relax - (I0 * drho + rho0 * dI))
    M[2, 1] += -ik * gam * p0
    # vibrational energy: E_t = -E_nu0 u_x + (E_nue - E_nu)/tau + rho Q
    M[3, :] += -relax + Q0 * drho + rho0 * dQ
    M[3, 1] += -ik * ev0
    return M


def omegas(gas, k):
    """The four roots omega(k) (complex), sorted by real part."""
    lam = np.linalg.eigvals(matrix(gas, k))
    om = 1j * lam
    return om[np.argsort(om.real)]


def modes(gas, k):
    """(omega, eigenvector) pairs, eigenvectors over (rho', u', p', E_nu')."""
    lam, V = np.linalg.eig(matrix(gas, k))
    return [(1j * l, V[:, i]) for i, l in enumerate(lam)]


def acoustic_mode(gas, k, direction=+1):
    """Right- (direction=+1) or left-going sound wave: the root with the
    largest |Re omega| of the given sign."""
    best = None
    for om, v in modes(gas, k):
        if np.sign(om.real) == direction and (best is None or abs(om.real) > abs(best[0].real)):
            best = (om, v)
    return best


def paper_residual(gas, omega, k):
    """LHS - RHS of eq. (8), each side scaled by k^2 c0^2 to be O(1)."""
    g = gas
    gam, gm1, R, T0 = g["gamma"], g["gamma"] - 1.0, g["R"], g["T0"]
    tau0, Q0, I0 = g["tau0"], g["Q0"], g["I0"]
    Ck = g["Cv"] / R
    S = tau0 * Q0 / (R * T0)
    c0sq = gam * R * T0
    d = omega * tau0
    A = 1.0 + (Ck + S * (g["tau_T"] + g["Q_T"])) * gm1
    B = 1.0 + (Ck + S * (g["tau_T"] - g["tau_rho"] + g["Q_T"] - g["Q_rho"])) * gm1 / gam
    lhs = omega ** 2 * ((A - 1j * d) + 1j * (1.0 - 1j * d) * gm1 / (omega * R * T0)
                        * (I0 * g["I_T"] - Q0 * g["Q_T"]))
    rhs = k ** 2 * c0sq * ((B - 1j * d) + 1j * (1.0 - 1j * d) * gm1 / (omega * gam * T0 * R)
                           * (I0 * (g["I_T"] - g["I_rho"]) - Q0 * (g["Q_T"] - g["Q_rho"])))
    return (lhs - rhs) / (k ** 2 * c0sq)


def S1(gas):
    """Lower threshold of negative dispersion printed after eq. (8)."""
    Ck = gas["Cv"] / gas["R"]
    gm1 = gas["gamma"] - 1.0
    return -gm1 * Ck / (gas["tau_rho"] + gm1 * gas["tau_T"])


def spatial_mode(gas, omega, direction=+1):
    """Signalling problem: the complex wavenumber k of a wave of real
    frequency omega, exp(-i omega t + i k x), travelling in the given
    direction (sign of Re k), and its eigenvector over (rho', u', p', E_nu')
    scaled to rho' = 1.  M(k) is affine in k, M = M0 + k M1, so k is a finite
    generalised eigenvalue of (-i omega I - M0) X = k M1 X; the amplitude then
    varies along x as exp(-Im k x)."""
    import scipy.linalg as sl
    M0 = matrix(gas, 0.0)
    M1 = matrix(gas, 1.0) - M0
    A = -1j * omega * np.eye(4) - M0
    ks, V = sl.eig(A, M1)
    idx = [i for i in range(len(ks)) if np.isfinite(ks[i]) and np.sign(ks[i].real) == direction]
    assert len(idx) == 1, ks
    i = idx[0]
    return complex(ks[i]), V[:, i] / V[0, i]


def spatial_k(gas, omega, direction=+1):
    return spatial_mode(gas, omega, direction)[0]


def source_transmission(gas, omega):
    """Complex amplitude (density, relative to the source's) of the
    right-going wave that a frozen plane sound wave imposed at x = 0 sets up in
    the medium: the wave entering through x = 0 carries the incoming frozen
    characteristic p' + rho0 c u' of the imposed state (2 c^2 per unit
    density amplitude), and the medium's mode must carry the same."""
    rho0, p0, _, _ = background(gas)
    c = np.sqrt(gas["gamma"] * p0 / rho0)
    _, X = spatial_mode(gas, omega)
    return 2.0 * c * c / (X[2] + rho0 * c * X[1])
