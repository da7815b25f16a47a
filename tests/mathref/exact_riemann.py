"""Exact solution of the Riemann problem for the ideal-gas Euler equations.

A pin for the oracle, independent of it: in the limit with no vibrational
energy (Cv = 0, so E_nue = 0 and E_nu stays 0) and no pump or sink, eqs.
(1)-(5) are the Euler equations of a gas with adiabatic exponent gamma, and a
piecewise-constant initial state has this self-similar solution.

Written from the mathematics: the star pressure solves
    f_L(p) + f_R(p) + (u_R - u_L) = 0,
where f_K is the Hugoniot velocity jump across a shock (p > p_K) or the
Riemann-invariant jump across a rarefaction (p <= p_K); the star velocity is
u* = (u_L + u_R)/2 + (f_R(p*) - f_L(p*))/2, and the solution at x/t is read
off the wave pattern.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.optimize import brentq


def _f(p, rho, pk, gamma):
    c = math.sqrt(gamma * pk / rho)
    if p > pk:
        A = 2.0 / ((gamma + 1.0) * rho)
        B = (gamma - 1.0) / (gamma + 1.0) * pk
        return (p - pk) * math.sqrt(A / (p + B))
    return 2.0 * c / (gamma - 1.0) * ((p / pk) ** ((gamma - 1.0) / (2.0 * gamma)) - 1.0)


def star_state(left, right, gamma):
    """left/right = (rho, u, p).  Returns dict(p, u, rho_L, rho_R, speeds)."""
    rL, uL, pL = left
    rR, uR, pR = right
    g = lambda p: _f(p, rL, pL, gamma) + _f(p, rR, pR, gamma) + (uR - uL)
    lo, hi = 1e-14, max(pL, pR)
    while g(hi) < 0.0:
        hi *= 2.0
    ps = brentq(g, lo, hi, xtol=1e-15, rtol=1e-15, maxiter=500)
    us = 0.5 * (uL + uR) + 0.5 * (_f(ps, rR, pR, gamma) - _f(ps, rL, pL, gamma))
    gm = (gamma - 1.0) / (gamma + 1.0)
    out = dict(p=ps, u=us)
    for side, (r, u, p), sgn in (("L", left, -1.0), ("R", right, 1.0)):
        c = math.sqrt(gamma * p / r)
        if ps > p:  # shock
            out["rho_" + side] = r * (ps / p + gm) / (gm * ps / p + 1.0)
            out["shock_" + side] = u + sgn * c * math.sqrt(
                (gamma + 1.0) / (2.0 * gamma) * ps / p + (gamma - 1.0) / (2.0 * gamma))
        else:  # rarefaction
            out["rho_" + side] = r * (ps / p) ** (1.0 / gamma)
            cs = c * (ps / p) ** ((gamma - 1.0) / (2.0 * gamma))
            out["head_" + side] = u + sgn * c
            out["tail_" + side] = us + sgn * cs
    return out


def sample(left, right, gamma, xi):
    """(rho, u, p) of the exact solution at similarity coordinates xi = x/t."""
    st = star_state(left, right, gamma)
    ps, us = st["p"], st["u"]
    xi = np.asarray(xi, dtype=np.float64)
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    p = np.empty_like(xi)
    for i, s in enumerate(xi.ravel()):
        if s <= us:
            r0, u0, p0 = left
            sgn = 1.0
            key = "L"
        else:
            r0, u0, p0 = right
            sgn = -1.0
            key = "R"
        c0 = math.sqrt(gamma * p0 / r0)
        if ps > p0:  # shock on this side
            S = st["shock_" + key]
            outside = s < S if key == "L" else s > S
            if outside:
                vals = (r0, u0, p0)
            else:
                vals = (st["rho_" + key], us, ps)
        else:
            head, tail = st["head_" + key], st["tail_" + key]
            if (key == "L" and s <= head) or (key == "R" and s >= head):
                vals = (r0, u0, p0)
            elif (key == "L" and s >= tail) or (key == "R" and s <= tail):
                vals = (st["rho_" + key], us, ps)
            else:  # inside the fan
                a = 2.0 / (gamma + 1.0)
                b = (gamma - 1.0) / ((gamma + 1.0) * c0)
                base = a + sgn * b * (u0 - s)
                vals = (r0 * base ** (2.0 / (gamma - 1.0)),
                        a * (sgn * c0 + (gamma - 1.0) / 2.0 * u0 + s),
                        p0 * base ** (2.0 * gamma / (gamma - 1.0)))
        rho.flat[i], u.flat[i], p.flat[i] = vals
    return rho, u, p
