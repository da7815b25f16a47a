// ng_csph.hpp -- per-particle and per-face FP64 arithmetic of the CSPH-TVD
// step (Khrapov & Khoperskov, arXiv:1805.03442, section 2.3, eqs. (9)-(14)),
// 1D.
//
// One particle per cell starts each step at the cell centre with the cell's
// conserved values (rho, rho u, E, E_nu).  The Lagrangian stage moves it with
// a predictor (eq. (10)) and a corrector (eq. (11)) under the right-hand side
// Y of eq. (12): the SPH pressure force and pressure work over the two
// neighbours, the body force, pump and sink of eqs. (2)-(3) and the E_nu
// source of eq. (4).  The Eulerian stage (eq. (9)) remaps the particles to
// the grid with the HLL flux (eq. (13)) of the advective F = u U between the
// face values of eq. (14), which take the particle's displacement xi into
// account.
//
// Readings where the text is silent or garbled: W is the cubic spline of
// smoothing length h (support 2h, 1D normalisation 2/(3h)) and the particle
// volume V = h; the leading minus of eq. (12) belongs to the two pressure
// terms; U^{n+1/2} of eq. (14) is the mean of U^n and the Lagrangian result;
// the slopes Theta are minmod-limited differences of U^n per unit length;
// the sources are explicit.
//
// Each formula is written in one fixed evaluation order and the library is
// built without multiply-add contraction, so that the FP64 results are the
// IEEE results of that order.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include "ng_cell.hpp"

namespace ng {

// d/dr_i of W(|d|, h) at d = r_i - r_j; wn = 2 / (3 h^2) (the 1D cubic
// spline's normalisation over h)
__device__ __forceinline__ double csph_grad_w(double d, double h, double wn)
{
    const double q = fabs(d) / h;
    double f;
    if (q < 1.0)
        f = -3.0 * q + 2.25 * (q * q);
    else if (q < 2.0)
        f = -0.75 * ((2.0 - q) * (2.0 - q));
    else
        f = 0.0;
    const double g = wn * f;
    return d > 0.0 ? g : (d < 0.0 ? -g : 0.0);
}

// velocity, pressure (eq. (5)) and phi = sqrt(2 p) of a particle's conserved
// values U = (rho, rho u, E, E_nu)
__device__ __forceinline__ void csph_prim(const K64& k, const double* U, double& u, double& p,
                                          double& phi)
{
    u = U[1] / U[0];
    p = k.gm1 * (U[2] - 0.5 * U[0] * (u * u) - U[3]);
    phi = sqrt(2.0 * p);
}

// Y of eq. (12) at a particle (rho, u, p, E_nu, phi) whose neighbours j-1 and
// j+1 have (phi_a, u_a) and (phi_b, u_b) and kernel gradients ga, gb; h is
// the particle volume.  sE and sV receive the source parts of the energy and
// E_nu rows (the budget).
__device__ __forceinline__ void csph_y(const K64& k, double h, double ga, double gb, double phia,
                                       double ua, double phib, double ub, double rho, double u,
                                       double p, double ev, double phi, double* Y, double& sE,
                                       double& sV)
{
    const double sp = phia * ga + phib * gb;
    const double se = phia * (0.5 * (u + ua)) * ga + phib * (0.5 * (u + ub)) * gb;
    const double T = p / (k.R * rho);
    double tau, Q, I;
    closures64(k, rho, T, tau, Q, I);
    const double Ee = rho * k.Cv * T;
    sE = rho * (u * k.fx + Q - I);
    sV = (Ee - ev) / tau + rho * Q;
    const double hp = -(h * phi);
    Y[0] = 0.0;
    Y[1] = hp * sp + rho * k.fx;
    Y[2] = hp * se + sE;
    Y[3] = sV;
}

// HLL flux (eq. (13)) of the advective F = u (rho, rho u, E, E_nu) between
// conserved face values UL and UR, with the wave speeds printed below it
__device__ __forceinline__ void csph_flux(const K64& k, const double* UL, const double* UR,
                                          double* F)
{
    const double uL = UL[1] / UL[0], uR = UR[1] / UR[0];
    const double pL = k.gm1 * (UL[2] - 0.5 * UL[0] * (uL * uL) - UL[3]);
    const double pR = k.gm1 * (UR[2] - 0.5 * UR[0] * (uR * uR) - UR[3]);
    const double cL = sqrt(k.gam * pL / UL[0]), cR = sqrt(k.gam * pR / UR[0]);
    const double SL = fmin(uL - cL, uR - cR);
    const double SR = fmax(uL + cL, uR + cR);
    const double SLR = SL * SR, dS = SR - SL;
    for (int c = 0; c < 4; c++) {
        const double fl = uL * UL[c], fr = uR * UR[c];
        if (0.0 < SL)
            F[c] = fl;
        else if (SR < 0.0)
            F[c] = fr;
        else
            F[c] = (SR * fl - SL * fr + SLR * (UR[c] - UL[c])) / dS;
    }
}

}  // namespace ng
