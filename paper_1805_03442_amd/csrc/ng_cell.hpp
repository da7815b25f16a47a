// ng_cell.hpp -- per-cell and per-face arithmetic of the MUSCL step for the
// vibrationally excited gas (Khrapov & Khoperskov, J. Phys.: Conf. Ser. 973
// (2018) 012007), in the two precisions of the library.
//
// FP64 ("Plain64"): the full conserved state U = (rho, rho u, rho v, E, E_nu)
// and the formulas exactly as eqs. (5), (13)-(15) state them, each written in
// one fixed evaluation order; the library is built without multiply-add
// contraction so that these are the IEEE results of that order.
//
// FP32 ("Dev32"): the state is stored as deviations from a uniform reference
// at rest, and the energy slot holds e = E - E_nu (the thermal and kinetic
// part) instead of E: (d rho, rho u, rho v, de = e - e_r, dEv = E_nu - Ev_r)
// with e_r = p_r/(gamma - 1).  Pressure then needs no difference of E and
// E_nu (eq. (5): p = (gamma - 1)(e - rho|v|^2/2)), so a medium whose E_nu lies
// far from the reference (the passive part of the sector run) keeps its
// pressure accurate.  e obeys the energy equation minus the E_nu equation:
// flux u (e + p), source rho (Q - I) + rho v.f minus the E_nu source.  Every
// flux and source is evaluated in a form in which the reference part cancels
// exactly:
//   p - p_r       = (gamma - 1)(de - rho|v|^2/2)                 (eq. (5))
//   F - F(U_ref)  = (rho u, rho u^2 + dp, rho u v, u (H_r + de + dp), u Ev),
//                   H_r = e_r + p_r
//   E_nue - E_nu  = (Cv/R) dp - dEv + (Cv/R p_r - Ev_r)          (eq. (7))
//   U*_K - U_K    = q_K (rho, rho S_K, rho v, e + p + rho (S_K - u) S*, Ev)_K,
//                   q_K = (S* - u_K)/(S_K - S*)                 (HLLC star jump)
// so that the O(1) background never enters a difference of two fluxes.  FP32
// rounding then acts on the perturbation, not on the background.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "ng_internal.hpp"

namespace ng {

// ------------------------------------------------------------- limiter

// minmod of two undivided differences (slopes of eq. (14)): zero unless both
// have the same strict sign, else the one of smaller magnitude.
__device__ __forceinline__ double minmod(double a, double b)
{
    if (a > 0.0 && b > 0.0) return a < b ? a : b;
    if (a < 0.0 && b < 0.0) return a > b ? a : b;
    return 0.0;
}
__device__ __forceinline__ float minmod(float a, float b)
{
    // the median of (a, b, 0) is exactly that selection
    return __builtin_amdgcn_fmed3f(a, b, 0.0f);
}

// ===================================================================== FP64

struct K64 {
    double gam, gm1, R, Cv, rho0, T0, tau0, tr, tT, Q0, Qr, QT, I0, Ir, IT, fx, fy;
    double stiff_z;
    double dt, dtdx, hdtdx, hdt;
    int riemann;
};

// pow for the exponents without a short form, kept out of line: the step
// kernels hold several closure evaluations, and inlined copies of pow would
// make their code many times larger than the path they run
__device__ __noinline__ double pow_general(double x, double a) { return pow(x, a); }

// x^a of the power laws (6): exponents 0, 1, -1, 2 and 1/2 by the correctly
// rounded IEEE operations (the exact power rounded once), others by pow.  The
// exponent is the same for every lane, so the selection is a scalar branch.
__device__ __forceinline__ double powr64(double x, double a)
{
    if (a == 0.0) return 1.0;
    if (a == 1.0) return x;
    if (a == -1.0) return 1.0 / x;
    if (a == 2.0) return x * x;
    if (a == 0.5) return sqrt(x);
    return pow_general(x, a);
}

// closures of eq. (6) at (rho, T); the predictor and corrector scale Q and I
// by act, 0 outside an active wedge (the 2D sector run of section 3)
__device__ __forceinline__ void closures64(const K64& k, double rho, double T, double& tau,
                                           double& Q, double& I)
{
    double r = rho / k.rho0, t = T / k.T0;
    tau = k.tau0 * powr64(r, k.tr) * powr64(t, k.tT);
    Q = k.Q0 * powr64(r, k.Qr) * powr64(t, k.QT);
    I = k.I0 * powr64(r, k.Ir) * powr64(t, k.IT);
}

// conserved -> primitive (eq. (5) solved for p); NC = 4 (1D) or 5 (2D)
template <int NC>
__device__ __forceinline__ void prim64(const K64& k, const double* U, double* W)
{
    double rho = U[0];
    double u = U[1] / rho;
    if (NC == 5) {
        double v = U[2] / rho;
        double ke = 0.5 * rho * (u * u + v * v);
        W[0] = rho;
        W[1] = u;
        W[2] = v;
        W[3] = k.gm1 * (U[3] - ke - U[4]);
        W[4] = U[4];
    } else {
        double ke = 0.5 * rho * (u * u);
        W[0] = rho;
        W[1] = u;
        W[2] = k.gm1 * (U[2] - ke - U[3]);
        W[3] = U[3];
    }
}

// signal speed of eq. (16): max(|v| + c, 2|v|)
template <int NC>
__device__ __forceinline__ double speed64(const K64& k, const double* W)
{
    double rho = W[0], u = W[1];
    double vel, p;
    if (NC == 5) {
        vel = sqrt(u * u + W[2] * W[2]);
        p = W[3];
    } else {
        vel = sqrt(u * u);
        p = W[2];
    }
    double c = sqrt(k.gam * p / rho);
    return fmax(vel + c, 2.0 * vel);
}

// Half-step predictor: quasi-linear primitive form of eqs. (1)-(5) with the
// sources at t^n (the "predictor" of the two-step scheme of section 2.3).
// W = (rho, u, v, p, E_nu) (2D) or (rho, u, p, E_nu) (1D); sx, sy limited slopes.
template <int NC>
__device__ __forceinline__ void predict64(const K64& k, const double* W, const double* sx,
                                          const double* sy, double* Wh, double act = 1.0)
{
    const double gam = k.gam, gm1 = k.gm1, hdtdx = k.hdtdx, hdt = k.hdt;
    if (NC == 5) {
        double rho = W[0], u = W[1], v = W[2], p = W[3], ev = W[4];
        double sr = sx[0], su = sx[1], sv = sx[2], sp = sx[3], se = sx[4];
        double ax_r = u * sr + rho * su;
        double ax_u = u * su + sp / rho;
        double ax_v = u * sv;
        double ax_p = u * sp + gam * p * su;
        double ax_e = u * se + ev * su;
        double tr = sy[0], tu = sy[1], tv = sy[2], tp = sy[3], te = sy[4];
        double ay_r = v * tr + rho * tv;
        double ay_u = v * tu;
        double ay_v = v * tv + tp / rho;
        double ay_p = v * tp + gam * p * tv;
        double ay_e = v * te + ev * tv;
        double T = p / (k.R * rho);
        double tau, Q, I;
        closures64(k, rho, T, tau, Q, I);
        Q = act * Q;
        I = act * I;
        double Ee = rho * k.Cv * T;
        Wh[0] = rho - hdtdx * (ax_r + ay_r);
        Wh[1] = u - hdtdx * (ax_u + ay_u) + hdt * k.fx;
        Wh[2] = v - hdtdx * (ax_v + ay_v) + hdt * k.fy;
        if (k.dt / tau > k.stiff_z) {
            // eq. (4) over dt/2 solved exactly with E_nue, tau, Q frozen
            double dEv = ((Ee + tau * (rho * Q)) - ev) * (-expm1(-(hdt / tau)));
            Wh[3] = p - hdtdx * (ax_p + ay_p) - gm1 * (dEv - hdt * (rho * (Q - I)));
            Wh[4] = ev - hdtdx * (ax_e + ay_e) + dEv;
        } else {
            double dEr = hdt * ((Ee - ev) / tau);
            Wh[3] = p - hdtdx * (ax_p + ay_p) - gm1 * (dEr + hdt * (rho * I));
            Wh[4] = ev - hdtdx * (ax_e + ay_e) + (dEr + hdt * (rho * Q));
        }
    } else {
        double rho = W[0], u = W[1], p = W[2], ev = W[3];
        double sr = sx[0], su = sx[1], sp = sx[2], se = sx[3];
        double ax_r = u * sr + rho * su;
        double ax_u = u * su + sp / rho;
        double ax_p = u * sp + gam * p * su;
        double ax_e = u * se + ev * su;
        double T = p / (k.R * rho);
        double tau, Q, I;
        closures64(k, rho, T, tau, Q, I);
        Q = act * Q;
        I = act * I;
        double Ee = rho * k.Cv * T;
        Wh[0] = rho - hdtdx * ax_r;
        Wh[1] = u - hdtdx * ax_u + hdt * k.fx;
        if (k.dt / tau > k.stiff_z) {
            double dEv = ((Ee + tau * (rho * Q)) - ev) * (-expm1(-(hdt / tau)));
            Wh[2] = p - hdtdx * ax_p - gm1 * (dEv - hdt * (rho * (Q - I)));
            Wh[3] = ev - hdtdx * ax_e + dEv;
        } else {
            double dEr = hdt * ((Ee - ev) / tau);
            Wh[2] = p - hdtdx * ax_p - gm1 * (dEr + hdt * (rho * I));
            Wh[3] = ev - hdtdx * ax_e + (dEr + hdt * (rho * Q));
        }
    }
}

// Interface flux along a normal.  Face states (rho, u_n, [u_t], p, E_nu);
// returns (mass, normal momentum, [tangential momentum], energy, E_nu) fluxes.
// HLL: eq. (13) with the wave speeds printed under it; HLLC: three waves, the
// middle one from equal pressure and normal velocity across the contact.
template <int NC, int RS>
__device__ __forceinline__ void flux64(const K64& k, const double* WL, const double* WR,
                                       double* F)
{
    const double gam = k.gam, gm1 = k.gm1;
    double rL = WL[0], uL = WL[1], rR = WR[0], uR = WR[1];
    double vL, vR, pL, pR, eL, eR, EL, ER;
    if (NC == 5) {
        vL = WL[2];
        vR = WR[2];
        pL = WL[3];
        pR = WR[3];
        eL = WL[4];
        eR = WR[4];
        EL = pL / gm1 + 0.5 * rL * (uL * uL + vL * vL) + eL;
        ER = pR / gm1 + 0.5 * rR * (uR * uR + vR * vR) + eR;
    } else {
        vL = vR = 0.0;
        pL = WL[2];
        pR = WR[2];
        eL = WL[3];
        eR = WR[3];
        EL = pL / gm1 + 0.5 * rL * (uL * uL) + eL;
        ER = pR / gm1 + 0.5 * rR * (uR * uR) + eR;
    }
    double mL = rL * uL, mR = rR * uR;
    // physical fluxes and conserved face states, component order (rho, m_n, [m_t], E, Ev)
    double FL[5], FR[5], UL[5], UR[5];
    FL[0] = mL;
    FL[1] = mL * uL + pL;
    FR[0] = mR;
    FR[1] = mR * uR + pR;
    UL[0] = rL;
    UL[1] = rL * uL;
    UR[0] = rR;
    UR[1] = rR * uR;
    const int iE = NC == 5 ? 3 : 2, iV = NC == 5 ? 4 : 3;
    if (NC == 5) {
        FL[2] = mL * vL;
        FR[2] = mR * vR;
        UL[2] = rL * vL;
        UR[2] = rR * vR;
    }
    FL[iE] = uL * (EL + pL);
    FR[iE] = uR * (ER + pR);
    FL[iV] = uL * eL;
    FR[iV] = uR * eR;
    UL[iE] = EL;
    UR[iE] = ER;
    UL[iV] = eL;
    UR[iV] = eR;

    double cL = sqrt(gam * pL / rL);
    double cR = sqrt(gam * pR / rR);
    double SL = fmin(uL - cL, uR - cR);
    double SR = fmax(uL + cL, uR + cR);

    if (RS == 1) {
        // HLL, eq. (13)
        double inv = SR - SL;
        for (int c = 0; c < NC; c++) {
            double fh = (SR * FL[c] - SL * FR[c] + SL * SR * (UR[c] - UL[c])) / inv;
            F[c] = (0.0 < SL) ? FL[c] : ((SR < 0.0) ? FR[c] : fh);
        }
        return;
    }
    double dL = SL - uL, dR = SR - uR;
    double Ss = (pR - pL + rL * uL * dL - rR * uR * dR) / (rL * dL - rR * dR);
    // the star state on the side of the contact that the face sees
    bool left = 0.0 < Ss;
    double rK = left ? rL : rR, uK = left ? uL : uR, vK = left ? vL : vR;
    double pK = left ? pL : pR, eK = left ? eL : eR, EK = left ? EL : ER;
    double SK = left ? SL : SR, dK = left ? dL : dR;
    double fac = rK * dK / (SK - Ss);
    double Us[5];
    Us[0] = fac;
    Us[1] = fac * Ss;
    if (NC == 5) Us[2] = fac * vK;
    Us[iE] = fac * (EK / rK + (Ss - uK) * (Ss + pK / (rK * dK)));
    Us[iV] = fac * (eK / rK);
    bool star = left || (0.0 <= SR);
    for (int c = 0; c < NC; c++) {
        double FK = left ? FL[c] : FR[c];
        double UK = left ? UL[c] : UR[c];
        double fs = FK + SK * (Us[c] - UK);
        F[c] = (0.0 < SL) ? FL[c] : (star ? fs : FR[c]);
    }
}

// Sources Y of eq. (15) at the half-step state and the conservative update.
// Un: conserved state at t^n; dF, dG: flux differences over the cell; Wh: the
// half-step primitive state.  Writes Unew and the cell's contributions to the
// source budget (dt * Y_E and the E_nu source increment).
template <int NC>
__device__ __forceinline__ void update64(const K64& k, const double* Un, const double* dF,
                                         const double* dG, const double* Wh, double* Unew,
                                         double& srcE, double& srcV, double act = 1.0)
{
    const double dt = k.dt, dtdx = k.dtdx;
    double rho = Wh[0], u = Wh[1];
    double v = 0.0, p, ev;
    if (NC == 5) {
        v = Wh[2];
        p = Wh[3];
        ev = Wh[4];
    } else {
        p = Wh[2];
        ev = Wh[3];
    }
    double T = p / (k.R * rho);
    double tau, Q, I;
    closures64(k, rho, T, tau, Q, I);
    Q = act * Q;
    I = act * I;
    double Ee = rho * k.Cv * T;
    double Y[5];
    const int iE = NC == 5 ? 3 : 2, iV = NC == 5 ? 4 : 3;
    Y[0] = 0.0;
    Y[1] = rho * k.fx;
    if (NC == 5) {
        Y[2] = rho * k.fy;
        Y[iE] = rho * (u * k.fx + v * k.fy + Q - I);
    } else {
        Y[iE] = rho * (u * k.fx + Q - I);
    }
    Y[iV] = (Ee - ev) / tau + rho * Q;
    for (int c = 0; c < NC; c++) {
        if (NC == 5)
            Unew[c] = Un[c] - dtdx * (dF[c] + dG[c]) + dt * Y[c];
        else
            Unew[c] = Un[c] - dtdx * dF[c] + dt * Y[c];
    }
    double de = dt * Y[iV];
    double z = dt / tau;
    if (z > k.stiff_z) {
        // eq. (4) over the whole step solved exactly from the start-of-step
        // E_nu, with E_nue, tau and Q frozen at t^{n+1/2}
        de = ((Ee + tau * (rho * Q)) - Un[iV]) * (-expm1(-z));
        if (NC == 5)
            Unew[iV] = Un[iV] - dtdx * (dF[iV] + dG[iV]) + de;
        else
            Unew[iV] = Un[iV] - dtdx * dF[iV] + de;
    }
    srcE = dt * Y[iE];
    srcV = de;
}

// ===================================================================== FP32

__device__ __forceinline__ float rcp32(float x) { return __builtin_amdgcn_rcpf(x); }

// Stiff branch: eq. (4) solved exactly over a time z tau with E_nue, tau and
// Q frozen, E_nu(z tau) - E_nu = (num + tau rhoQ)(1 - exp(-z)), num = E_nue -
// E_nu, evaluated in FP64 and returned less hq (the caller's explicit pump
// term, which it adds back).  Kept out of line: it runs only where dt/tau is
// large.
__device__ __noinline__ float relax_exact(float num, float rhoQ, float itau, double z, float hq)
{
    const double a = ((double)num + (double)rhoQ / (double)itau) * (-expm1(-z));
    return (float)(a - (double)hq);
}

struct K32 {
    float gam, gm1, igm1, CvR;
    float rho_r, p_r, ev_r, H_r, D_r;   // reference state and its cancelled constants
                                        // (H_r = e_r + p_r, e = E - E_nu)
    float cl_c[3], cl_a[3], cl_b[3];    // closures of eq. (6): c rho^a p^b
    float fx, fy;
    float gp_r;                         // gamma p_r
    float stiff_z, hstiff_z;            // stiffness threshold on dt/tau, and half of it
    float dt, dtdx, hdtdx, hdt;
    float hdtfx, hdtfy;                 // (dt/2) f, the body force of the predictor
    double dt64, hdt64;
    int riemann;
    bool force;                         // f != 0
};

// x^(C/2) for a half-integer exponent code C in [-4, 4] known at compile
// time, from x, 1/x and 1/sqrt(x)
template <int C>
__device__ __forceinline__ float pw_half(float x, float ix, float sx)
{
    static_assert(C >= -4 && C <= 4, "exponent code out of range");
    if constexpr (C == 0) return 1.0f;
    else if constexpr (C == 1) return x * sx;
    else if constexpr (C == 2) return x;
    else if constexpr (C == 3) return x * (x * sx);
    else if constexpr (C == 4) return x * x;
    else if constexpr (C == -1) return sx;
    else if constexpr (C == -2) return ix;
    else if constexpr (C == -3) return ix * sx;
    else return ix * ix;
}

// 1/tau, Q and I of eq. (6) at full (rho, p) in FP32, each c rho^a p^b
// (T = p / (R rho)).  Recipe CL > 0 (kRecipeCodes): the half-integer
// exponents are compile-time constants, so each power is a product of rho,
// p, 1/rho, 1/p and reciprocal square roots (at most one transcendental per
// base).  CL = 0: one exp2 of a log2(rho) + b log2(p) per closure.  HaveIr:
// irho is 1/rho; otherwise it is computed here when an exponent needs it.
template <bool HaveIr, int CL>
__device__ __forceinline__ void closures32(const K32& k, float rho, float p, float irho,
                                           float& itau, float& Q, float& I)
{
    if constexpr (CL == 0) {
        const float lr = __builtin_amdgcn_logf(rho), lp = __builtin_amdgcn_logf(p);
        itau = k.cl_c[0] * __builtin_amdgcn_exp2f(fmaf(k.cl_a[0], lr, k.cl_b[0] * lp));
        Q = k.cl_c[1] * __builtin_amdgcn_exp2f(fmaf(k.cl_a[1], lr, k.cl_b[1] * lp));
        I = k.cl_c[2] * __builtin_amdgcn_exp2f(fmaf(k.cl_a[2], lr, k.cl_b[2] * lp));
    } else {
        constexpr int a0 = kRecipeCodes[CL][0], b0 = kRecipeCodes[CL][1];
        constexpr int a1 = kRecipeCodes[CL][2], b1 = kRecipeCodes[CL][3];
        constexpr int a2 = kRecipeCodes[CL][4], b2 = kRecipeCodes[CL][5];
        constexpr bool odd_r = ((a0 | a1 | a2) & 1) != 0, neg_r = a0 < 0 || a1 < 0 || a2 < 0;
        constexpr bool odd_p = ((b0 | b1 | b2) & 1) != 0, neg_p = b0 < -1 || b1 < -1 || b2 < -1;
        float sr = 1.0f, ir = irho, ip = 1.0f, sp = 1.0f;
        if constexpr (odd_r) sr = __builtin_amdgcn_rsqf(rho);
        if constexpr (!HaveIr && neg_r) ir = odd_r ? sr * sr : rcp32(rho);
        if constexpr (neg_p) ip = rcp32(p);
        if constexpr (odd_p) sp = __builtin_amdgcn_rsqf(p);
        itau = k.cl_c[0] * (pw_half<a0>(rho, ir, sr) * pw_half<b0>(p, ip, sp));
        Q = k.cl_c[1] * (pw_half<a1>(rho, ir, sr) * pw_half<b1>(p, ip, sp));
        I = k.cl_c[2] * (pw_half<a2>(rho, ir, sr) * pw_half<b2>(p, ip, sp));
    }
}

// deviation primitives (d rho, u, [v], dp, dEv) from deviation conserved,
// and 1/rho in W[NC] for the predictor and the signal speed; rho |v|^2 is
// formed as m.v, the momentum times the velocity
template <int NC>
__device__ __forceinline__ void prim32(const K32& k, const float* D, float* W)
{
    float rho = k.rho_r + D[0];
    float ir = rcp32(rho);
    float u = D[1] * ir;
    W[NC] = ir;
    W[0] = D[0];
    W[1] = u;
    if (NC == 5) {
        float v = D[2] * ir;
        float m2 = fmaf(D[1], u, D[2] * v);
        W[2] = v;
        W[3] = k.gm1 * fmaf(-0.5f, m2, D[3]);
        W[4] = D[4];
    } else {
        W[2] = k.gm1 * fmaf(-0.5f, D[1] * u, D[2]);
        W[3] = D[3];
    }
}

// signal speed of eq. (16) in FP32, max(|v| + c, 2|v|) = |v| + max(c, |v|)
// (the same rounded value); c = sqrt(gamma p / rho) from the 1/rho that prim32
// leaves in W[NC]; square roots by the hardware (about 1 ulp; the speed only
// bounds dt)
template <int NC>
__device__ __forceinline__ float speed32(const K32& k, const float* W)
{
    float u = W[1];
    float v2 = NC == 5 ? W[2] * W[2] : 0.0f;
    float gp = fmaf(k.gam, W[NC == 5 ? 3 : 2], k.gp_r);
    float vel = __builtin_amdgcn_sqrtf(fmaf(u, u, v2));
    float c = __builtin_amdgcn_sqrtf(gp * W[NC]);
    return vel + fmaxf(c, vel);
}

// half-step predictor in primitive form: W + (dt/2)(-A_x dW/dx - A_y dW/dy + S(W))
// with undivided slopes sx, sy and the divergence su + tv shared by the
// density, pressure and E_nu rows.  FullRho: Wh[0] is the full density (the
// HLLC flux and the corrector use only that), else its deviation.
template <int NC, bool FullRho = false, int CL = 0>
__device__ __forceinline__ void predict32(const K32& k, const float* W, const float* sx,
                                          const float* sy, float* Wh, float act = 1.0f)
{
    const float hdtdx = k.hdtdx, hdt = k.hdt;
    constexpr int iP = NC == 5 ? 3 : 2, iV = NC == 5 ? 4 : 3;
    float dr = W[0], u = W[1], dp = W[iP], de = W[iV];
    float rho = k.rho_r + dr, p = k.p_r + dp, ev = k.ev_r + de;
    float irho = W[NC];
    float gp = fmaf(k.gam, dp, k.gp_r);
    float sr = sx[0], su = sx[1], sp = sx[iP], se = sx[iV];
    float a_r, a_u, a_v = 0.0f, a_p, a_e, v = 0.0f;
    if (NC == 5) {
        v = W[2];
        float sv = sx[2];
        float tr = sy[0], tu = sy[1], tv = sy[2], tp = sy[3], te = sy[4];
        float dv = su + tv;
        a_r = fmaf(u, sr, fmaf(v, tr, rho * dv));
        a_u = fmaf(u, su, fmaf(v, tu, sp * irho));
        a_v = fmaf(u, sv, fmaf(v, tv, tp * irho));
        a_p = fmaf(u, sp, fmaf(v, tp, gp * dv));
        a_e = fmaf(u, se, fmaf(v, te, ev * dv));
    } else {
        a_r = fmaf(u, sr, rho * su);
        a_u = fmaf(u, su, sp * irho);
        a_p = fmaf(u, sp, gp * su);
        a_e = fmaf(u, se, ev * su);
    }
    float itau, Q, I;
    closures32<true, CL>(k, rho, p, irho, itau, Q, I);
    Q = act * Q;
    I = act * I;
    float relax_num = fmaf(k.CvR, dp, k.D_r - de);   // E_nue - E_nu
    // (dt/2)/tau against half the threshold: the same decision as dt/tau
    // against the threshold (both sides scaled by exactly 1/2)
    float z = hdt * itau;
    float dEr;
    if (z > k.hstiff_z)
        dEr = relax_exact(relax_num, rho * Q, itau, k.hdt64 * (double)itau, hdt * (rho * Q));
    else
        dEr = relax_num * z;
    Wh[0] = fmaf(-hdtdx, a_r, FullRho ? rho : dr);
    Wh[1] = fmaf(-hdtdx, a_u, u);
    if (NC == 5) Wh[2] = fmaf(-hdtdx, a_v, v);
    if (k.force) {
        Wh[1] += k.hdtfx;
        if (NC == 5) Wh[2] += k.hdtfy;
    }
    Wh[iP] = fmaf(-k.gm1, fmaf(hdt, rho * I, dEr), fmaf(-hdtdx, a_p, dp));
    Wh[iV] = fmaf(hdt, rho * Q, dEr) + fmaf(-hdtdx, a_e, de);
}

// Interface flux minus the flux of the reference state, face states in
// deviation primitives.  HLLC is evaluated on one side only: the side K whose
// flux the face takes (L if 0 < S_L or 0 < S*, else R) gives
// F = F_K + S_K (U*_K - U_K), with the star jump zero on supersonic faces.
// With sq = S_K q_K the components factor as
//   rho (u + sq) = F_rho,  F_rho v,  (E + p)(u + sq) + sq rho (S_K - u) S*,
//   E_nu (u + sq).
// The HLLC flux takes face states with the full density in [0] (it uses the
// density only in products), HLL the deviation (its jump U_R - U_L).
template <int NC, int RS>
__device__ __forceinline__ void flux32(const K32& k, const float* WL, const float* WR, float* F)
{
    constexpr int iP = NC == 5 ? 3 : 2, iV = NC == 5 ? 4 : 3;
    float rL = RS == 1 ? k.rho_r + WL[0] : WL[0], rR = RS == 1 ? k.rho_r + WR[0] : WR[0];
    float uL = WL[1], uR = WR[1];
    float dpL = WL[iP], dpR = WR[iP];
    float gpL = fmaf(k.gam, dpL, k.gp_r), gpR = fmaf(k.gam, dpR, k.gp_r);
    float cL = gpL * __builtin_amdgcn_rsqf(gpL * rL);
    float cR = gpR * __builtin_amdgcn_rsqf(gpR * rR);
    float SL = fminf(uL - cL, uR - cR);
    float SR = fmaxf(uL + cL, uR + cR);
    float mL = rL * uL, mR = rR * uR;
    if (RS == 1) {
        // HLL, eq. (13), with both physical fluxes
        float vL = NC == 5 ? WL[2] : 0.0f, vR = NC == 5 ? WR[2] : 0.0f;
        float deL = WL[iV], deR = WR[iV];
        float m2L = NC == 5 ? fmaf(mL, uL, (rL * vL) * vL) : mL * uL;
        float m2R = NC == 5 ? fmaf(mR, uR, (rR * vR) * vR) : mR * uR;
        float dEL = fmaf(0.5f, m2L, dpL * k.igm1);   // de = e - e_r
        float dER = fmaf(0.5f, m2R, dpR * k.igm1);
        float HL = k.H_r + (dEL + dpL), HR = k.H_r + (dER + dpR);
        float UL[5], UR[5], FL[5], FR[5];
        UL[0] = WL[0];
        UR[0] = WR[0];
        UL[1] = mL;
        UR[1] = mR;
        FL[0] = mL;
        FR[0] = mR;
        FL[1] = fmaf(mL, uL, dpL);
        FR[1] = fmaf(mR, uR, dpR);
        if (NC == 5) {
            UL[2] = rL * vL;
            UR[2] = rR * vR;
            FL[2] = mL * vL;
            FR[2] = mR * vR;
        }
        UL[iP] = dEL;
        UR[iP] = dER;
        UL[iV] = deL;
        UR[iV] = deR;
        FL[iP] = uL * HL;
        FR[iP] = uR * HR;
        FL[iV] = uL * (k.ev_r + deL);
        FR[iV] = uR * (k.ev_r + deR);
        float inv = rcp32(SR - SL);
        float SLR = SL * SR;
        for (int c = 0; c < NC; c++) {
            float fh = fmaf(SLR, UR[c] - UL[c], fmaf(SR, FL[c], -(SL * FR[c]))) * inv;
            F[c] = (0.0f < SL) ? FL[c] : ((SR < 0.0f) ? FR[c] : fh);
        }
        return;
    }
    float dL = SL - uL, dR = SR - uR;
    float Ss = fmaf(mL, dL, fmaf(-mR, dR, dpR - dpL)) * rcp32(fmaf(rL, dL, -(rR * dR)));
    // bitwise on the comparison masks (no branch)
    const bool supL = 0.0f < SL, supR = SR < 0.0f;
    const bool left = supL | (!supR & (0.0f < Ss));
    float rK = left ? rL : rR, uK = left ? uL : uR, dpK = left ? dpL : dpR;
    float deK = left ? WL[iV] : WR[iV];
    float vK = NC == 5 ? (left ? WL[2] : WR[2]) : 0.0f;
    float SK = left ? SL : SR, dK = left ? dL : dR, mK = left ? mL : mR;
    float m2K = NC == 5 ? fmaf(mK, uK, (rK * vK) * vK) : mK * uK;   // rho |v|^2
    float dEK = fmaf(0.5f, m2K, dpK * k.igm1);   // de = e - e_r
    float HK = k.H_r + (dEK + dpK);   // e + p
    float evK = k.ev_r + deK;
    float q = (supL | supR) ? 0.0f : (Ss - uK) * rcp32(SK - Ss);
    float sq = SK * q, sqr = sq * rK;
    float us = uK + sq;
    float F0 = fmaf(sq, rK, mK);
    F[0] = F0;
    F[1] = fmaf(sqr, SK, fmaf(mK, uK, dpK));
    if (NC == 5) F[2] = F0 * vK;
    F[iP] = fmaf(HK, us, sqr * (dK * Ss));
    F[iV] = evK * us;
}

// corrector of eq. (15): U^n - dt/h (dF + dG) + dt Y(W^{n+1/2}); the source
// rows without a body force reduce to rho (Q - I) and (E_nue - E_nu)/tau + rho Q
template <int NC, bool FullRho = false, int CL = 0>
__device__ __forceinline__ void update32(const K32& k, const float* Un, const float* dF,
                                         const float* dG, const float* Wh, float* Unew,
                                         float& srcE, float& srcV, float act = 1.0f)
{
    constexpr int iP = NC == 5 ? 3 : 2, iV = NC == 5 ? 4 : 3;
    const float dt = k.dt, dtdx = k.dtdx;
    float u = Wh[1], dp = Wh[iP], de = Wh[iV];
    float v = NC == 5 ? Wh[2] : 0.0f;
    float rho = FullRho ? Wh[0] : k.rho_r + Wh[0], p = k.p_r + dp;
    float itau, Q, I;
    closures32<false, CL>(k, rho, p, 0.0f, itau, Q, I);
    Q = act * Q;
    I = act * I;
    float yE = rho * (Q - I);
    float relax_num = fmaf(k.CvR, dp, k.D_r - de);
    float yV = fmaf(relax_num, itau, rho * Q);
    float div[NC];
    for (int c = 0; c < NC; c++) div[c] = NC == 5 ? dF[c] + dG[c] : dF[c];
    for (int c = 0; c < NC; c++) Unew[c] = fmaf(-dtdx, div[c], Un[c]);
    if (k.force) {
        Unew[1] = fmaf(dt, rho * k.fx, Unew[1]);
        if (NC == 5) Unew[2] = fmaf(dt, rho * k.fy, Unew[2]);
        yE = fmaf(rho, fmaf(u, k.fx, v * k.fy), yE);
    }
    float dv = dt * yV;
    if (k.dt * itau > k.stiff_z) {
        // eq. (4) solved exactly from the start-of-step E_nu, FP64 factor
        float num = fmaf(k.CvR, dp, k.D_r - Un[iV]);
        float dEr = relax_exact(num, rho * Q, itau, k.dt64 * (double)itau, dt * (rho * Q));
        dv = fmaf(dt, rho * Q, dEr);
        Unew[iV] = dv + Unew[iV];
    } else {
        Unew[iV] = fmaf(dt, yV, Unew[iV]);
    }
    // e = E - E_nu gains the energy source less what E_nu gains
    Unew[iP] = fmaf(dt, yE, Unew[iP]) - dv;
    srcE = dt * yE;
    srcV = dv;
}

// The change of one step, -dt/h (dF + dG) + dt Y(W^{n+1/2}) (eq. (15)), for a
// state kept in another precision: the same sources and stiff branch as
// update32; ev_n is the start-of-step E_nu deviation the stiff branch relaxes.
template <int NC, bool FullRho = false, int CL = 0>
__device__ __forceinline__ void increment32(const K32& k, float ev_n, const float* dF,
                                            const float* dG, const float* Wh, float* dU,
                                            float& srcE, float& srcV, float act = 1.0f)
{
    constexpr int iP = NC == 5 ? 3 : 2, iV = NC == 5 ? 4 : 3;
    const float dt = k.dt, dtdx = k.dtdx;
    float u = Wh[1], dp = Wh[iP], de = Wh[iV];
    float v = NC == 5 ? Wh[2] : 0.0f;
    float rho = FullRho ? Wh[0] : k.rho_r + Wh[0], p = k.p_r + dp;
    float itau, Q, I;
    closures32<false, CL>(k, rho, p, 0.0f, itau, Q, I);
    Q = act * Q;
    I = act * I;
    float yE = rho * (Q - I);
    float relax_num = fmaf(k.CvR, dp, k.D_r - de);
    float yV = fmaf(relax_num, itau, rho * Q);
    for (int c = 0; c < NC; c++) dU[c] = -dtdx * (NC == 5 ? dF[c] + dG[c] : dF[c]);
    if (k.force) {
        dU[1] = fmaf(dt, rho * k.fx, dU[1]);
        if (NC == 5) dU[2] = fmaf(dt, rho * k.fy, dU[2]);
        yE = fmaf(rho, fmaf(u, k.fx, v * k.fy), yE);
    }
    float dv = dt * yV;
    if (k.dt * itau > k.stiff_z) {
        float num = fmaf(k.CvR, dp, k.D_r - ev_n);
        float dEr = relax_exact(num, rho * Q, itau, k.dt64 * (double)itau, dt * (rho * Q));
        dv = fmaf(dt, rho * Q, dEr);
        dU[iV] = dv + dU[iV];
    } else {
        dU[iV] = fmaf(dt, yV, dU[iV]);
    }
    dU[iP] = fmaf(dt, yE, dU[iP]) - dv;
    srcE = dt * yE;
    srcV = dv;
}

}  // namespace ng
