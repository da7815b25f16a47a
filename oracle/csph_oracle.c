/*
 * csph_oracle.c -- serial FP64 CPU oracle for the CSPH-TVD step of Khrapov &
 * Khoperskov (arXiv:1805.03442), section 2.3, eqs. (9)-(14), in 1D.
 *
 * TEST INFRASTRUCTURE. Only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark load this file. The product path (the HIP library) shares
 * no code with it and never calls it.
 *
 * It includes the MUSCL oracle for what the two schemes share: the gas model
 * (closures (6), EOS (7), conversions (5)), the time step of eq. (16) and the
 * ghost-cell rule of the boundary kinds.
 *
 * What one step n -> n+1 with a given dt computes, in the paper's order:
 *
 *   Lagrangian stage (eqs. (10)-(12)).  A "liquid" particle sits at the centre
 *   x_j of every cell at t^n and carries the cell's conserved values U_j =
 *   (rho, rho u, E, E_nu).  A predictor and a corrector advance them,
 *
 *     U*      = U^n + dt Y(U^n, r^n),           r*      = r^n + dt (u^n + u*)/2,
 *     U~^{n+1} = (U^n + U*)/2 + dt/2 Y(U*, r*),  r^{n+1} = (r^n + r*)/2
 *                                                        + dt/2 (u^n + u~^{n+1})/2,
 *
 *   with Y of eq. (12): no mass source; the SPH pressure force
 *   -V phi_j sum_j' phi_j' dW/dr_j and pressure work -V phi_j sum_j' phi_j'
 *   (u_j + u_j')/2 dW/dr_j over the neighbours j' = j-1, j+1 (phi = sqrt(2p),
 *   W(|r_j - r_j'|, h) the smoothing kernel, V = h the particle's volume); the
 *   body force, pump and sink as in eqs. (2)-(3); and the E_nu source of
 *   eq. (4).  Positions are kept as displacements xi = r - x from the cell
 *   centres (exactly the paper's r in exact arithmetic), so a distance is
 *   (j - j') h + (xi_j - xi_j').
 *
 *   Eulerian stage (eqs. (9), (13), (14)).  U^{n+1}_j = U~^{n+1}_j -
 *   dt/h (F_{j+1/2} - F_{j-1/2}) with the advective flux F = u (rho, rho u, E,
 *   E_nu) of eq. (9), HLL (eq. (13)) with the wave speeds printed below it,
 *   between the face values of eq. (14):
 *
 *     U^L = U^{n+1/2}_j     + (h - xi^{n+1}_j) Theta_j / 2,
 *     U^R = U^{n+1/2}_{j+1} - (h + xi^{n+1}_{j+1}) Theta_{j+1} / 2,
 *
 *   the values of each particle's linear profile, displaced with it, averaged
 *   over the slab that crosses the face.
 *
 * Readings (the paper is silent or garbled; DESIGN lists them):
 *   - W: the cubic spline of smoothing length h (support 2h), 1D
 *     normalisation 2/(3h); with V = h the sum gives dp/dx exactly to second
 *     order on the uniform lattice.
 *   - Signs of eq. (12): the leading minus belongs to the pressure terms; the
 *     body force, pump, sink and relaxation enter with the signs of eqs.
 *     (1)-(4), as in the MUSCL source Y (the relaxation in the form of eq.
 *     (4), (E_nue - E_nu)/tau + rho Q).
 *   - U^{n+1/2} of eq. (14) is (U^n + U~^{n+1})/2.
 *   - Theta: minmod-limited slopes of the conserved values at t^n, per unit
 *     length (the limiter the MUSCL oracle takes).
 *   - Boundaries: the ghost particles are the ghost cells of the MUSCL rule
 *     (periodic image, or mirror with the normal momentum reversed; before a
 *     forced source, the three particles x = -h/2, -3h/2, -5h/2 carry the
 *     source's plane wave at the step's start time, or_source_ghost); a
 *     ghost's displacement follows from its own velocity like any particle's.
 *   - No stiff branch: the sources are explicit in both stages.
 *
 * Layout as in muscl_oracle.c, 1D only: U[c * nx + j], c = 0..4 -> (rho,
 * rho u, rho v, E, E_nu) with rho v = 0.
 */
#include "muscl_oracle.c"

/* d/dr_j of the cubic-spline kernel W(|d|, h), d = r_j - r_j' (1D) */
static double cs_grad_w(double d, double h)
{
    double q = fabs(d) / h;
    double f;
    if (q < 1.0)
        f = -3.0 * q + 2.25 * (q * q);
    else if (q < 2.0)
        f = -0.75 * ((2.0 - q) * (2.0 - q));
    else
        f = 0.0;
    double g = (2.0 / (3.0 * (h * h))) * f;
    return d > 0.0 ? g : (d < 0.0 ? -g : 0.0);
}

/* The state of one particle as the Lagrangian stage needs it. */
typedef struct {
    double rho, m, E, ev;   /* conserved values                       */
    double u, p, phi;       /* velocity, pressure, sqrt(2 p)          */
    double xi;              /* displacement from the cell centre      */
} cs_part;

static void cs_fill(const or_gas* g, const double U[4], double xi, cs_part* P)
{
    double gm1 = g->gamma - 1.0;
    P->rho = U[0];
    P->m = U[1];
    P->E = U[2];
    P->ev = U[3];
    P->u = U[1] / U[0];
    P->p = gm1 * (U[2] - 0.5 * U[0] * (P->u * P->u) - U[3]);
    P->phi = sqrt(2.0 * P->p);
    P->xi = xi;
}

/* Y of eq. (12) for particle j with neighbours a = j-1 and b = j+1 (in that
 * order); act scales the pump and sink (the medium's activity).  yE and yV
 * receive the source parts of the energy and E_nu rows (the budget). */
static void cs_y(const or_gas* g, double h, const cs_part* a, const cs_part* c,
                 const cs_part* b, double act, double Y[4], double* yE, double* yV)
{
    /* distances r_j - r_j' as (j - j') h + (xi_j - xi_j') */
    double da = h + (c->xi - a->xi);
    double db = -h + (c->xi - b->xi);
    double ga = cs_grad_w(da, h), gb = cs_grad_w(db, h);
    double sp = a->phi * ga + b->phi * gb;
    double se = a->phi * (0.5 * (c->u + a->u)) * ga + b->phi * (0.5 * (c->u + b->u)) * gb;
    double T = c->p / (g->R * c->rho);
    double tau = or_tau(g, c->rho, T);
    double Q = act * or_Q(g, c->rho, T);
    double I = act * or_I(g, c->rho, T);
    double Ee = c->rho * g->Cv * T;
    double s_e = c->rho * (c->u * g->fx + Q - I);
    double s_v = (Ee - c->ev) / tau + c->rho * Q;
    Y[0] = 0.0;
    Y[1] = -(h * c->phi) * sp + c->rho * g->fx;
    Y[2] = -(h * c->phi) * se + s_e;
    Y[3] = s_v;
    *yE = s_e;
    *yV = s_v;
}

/* HLL flux (eq. (13)) of the advective F = u (rho, rho u, E, E_nu) between
 * conserved face values UL, UR */
static void cs_flux(const or_gas* g, const double UL[4], const double UR[4], double F[4])
{
    double gam = g->gamma, gm1 = gam - 1.0;
    double uL = UL[1] / UL[0], uR = UR[1] / UR[0];
    double pL = gm1 * (UL[2] - 0.5 * UL[0] * (uL * uL) - UL[3]);
    double pR = gm1 * (UR[2] - 0.5 * UR[0] * (uR * uR) - UR[3]);
    double cL = sqrt(gam * pL / UL[0]), cR = sqrt(gam * pR / UR[0]);
    double SL = fmin(uL - cL, uR - cR);
    double SR = fmax(uL + cL, uR + cR);
    int c;
    for (c = 0; c < 4; c++) {
        double fl = uL * UL[c], fr = uR * UR[c];
        if (0.0 < SL)
            F[c] = fl;
        else if (SR < 0.0)
            F[c] = fr;
        else
            F[c] = (SR * fl - SL * fr + SL * SR * (UR[c] - UL[c])) / (SR - SL);
    }
}

/*
 * One CSPH-TVD step from U_in (1D, ny = 1, 5 planes with rho v = 0), the state
 * at time t, to U_out with a given dt.  src[0] receives the energy sources of the step
 * (dt/2 of the predictor's plus dt/2 of the corrector's, summed over cells)
 * and src[1] those of E_nu.  xi_out, when not NULL, receives the n
 * displacements xi^{n+1} the Lagrangian stage leaves.  Returns OR_OK, or OR_EPHYS if a density or
 * pressure of U_out is not positive or a value is not finite; OR_EINVAL for a
 * 2D grid.
 */
int cs_step(const or_gas* g, const or_grid* gr, const or_num* nm, const double* U_in,
            double* U_out, double t, double dt, double* src, double* xi_out)
{
    (void)nm;
    if (gr->ny != 1) return OR_EINVAL;
    const int64_t n = gr->nx;
    const int64_t G = 3;                 /* stencil radius of the step    */
    const int64_t ne = n + 2 * G;
    const double h = gr->h;
    const double hdt = 0.5 * dt;
    const double dtdx = dt / h;
    /* extended arrays, index j + G for j = -G .. n + G - 1 */
    double* Un = (double*)calloc((size_t)(4 * ne), sizeof(double));
    double* Us = (double*)calloc((size_t)(4 * ne), sizeof(double));
    double* Ut = (double*)calloc((size_t)(4 * ne), sizeof(double));
    double* xs = (double*)calloc((size_t)ne, sizeof(double));
    double* xt = (double*)calloc((size_t)ne, sizeof(double));
    double* un = (double*)calloc((size_t)ne, sizeof(double));
    double* F = (double*)calloc((size_t)(4 * ne), sizeof(double));
    double* yE = (double*)calloc((size_t)ne, sizeof(double));
    double* yV = (double*)calloc((size_t)ne, sizeof(double));
    int64_t j;
    int c;
#define AT(A, c, j) (A)[(c) * ne + (j) + G]

    /* particles at the cell centres with the cell values (ghosts by the
     * boundary rule; a wall ghost carries the reversed momentum, a source
     * ghost the forced wave at time t) */
    for (j = -G; j < n + G; j++) {
        int flip;
        int64_t s = or_ghost(j, n, gr->bc[0], gr->bc[1], &flip);
        if (j < 0 && gr->bc[0] == OR_BC_SOURCE) {
            double Ug[5];
            or_source_ghost(g, gr, t, j, 0, Ug);
            AT(Un, 0, j) = Ug[0];
            AT(Un, 1, j) = Ug[1];
            AT(Un, 2, j) = Ug[3];
            AT(Un, 3, j) = Ug[4];
        } else {
            AT(Un, 0, j) = U_in[s];
            AT(Un, 1, j) = flip ? -U_in[n + s] : U_in[n + s];
            AT(Un, 2, j) = U_in[3 * n + s];
            AT(Un, 3, j) = U_in[4 * n + s];
        }
        un[j + G] = AT(Un, 1, j) / AT(Un, 0, j);
    }

    /* predictor, eq. (10), on particles -2 .. n+1 */
    for (j = -G + 1; j < n + G - 1; j++) {
        cs_part a, c0, b;
        double U[4], Y[4], se, sv;
        for (c = 0; c < 4; c++) U[c] = AT(Un, c, j - 1);
        cs_fill(g, U, 0.0, &a);
        for (c = 0; c < 4; c++) U[c] = AT(Un, c, j);
        cs_fill(g, U, 0.0, &c0);
        for (c = 0; c < 4; c++) U[c] = AT(Un, c, j + 1);
        cs_fill(g, U, 0.0, &b);
        cs_y(g, h, &a, &c0, &b, 1.0, Y, &se, &sv);
        for (c = 0; c < 4; c++) AT(Us, c, j) = AT(Un, c, j) + dt * Y[c];
        double us = AT(Us, 1, j) / AT(Us, 0, j);
        xs[j + G] = dt * (0.5 * (un[j + G] + us));
        yE[j + G] = hdt * se;
        yV[j + G] = hdt * sv;
    }

    /* corrector, eq. (11), on particles -1 .. n */
    for (j = -G + 2; j < n + G - 2; j++) {
        cs_part a, c0, b;
        double U[4], Y[4], se, sv;
        for (c = 0; c < 4; c++) U[c] = AT(Us, c, j - 1);
        cs_fill(g, U, xs[j - 1 + G], &a);
        for (c = 0; c < 4; c++) U[c] = AT(Us, c, j);
        cs_fill(g, U, xs[j + G], &c0);
        for (c = 0; c < 4; c++) U[c] = AT(Us, c, j + 1);
        cs_fill(g, U, xs[j + 1 + G], &b);
        cs_y(g, h, &a, &c0, &b, 1.0, Y, &se, &sv);
        for (c = 0; c < 4; c++)
            AT(Ut, c, j) = 0.5 * (AT(Un, c, j) + AT(Us, c, j)) + hdt * Y[c];
        double ut = AT(Ut, 1, j) / AT(Ut, 0, j);
        xt[j + G] = 0.5 * xs[j + G] + hdt * (0.5 * (un[j + G] + ut));
        yE[j + G] += hdt * se;
        yV[j + G] += hdt * sv;
    }

    /* faces j+1/2 for j = -1 .. n-1: slopes of U^n, face values of the
     * displaced profiles at t^{n+1/2}, HLL */
    for (j = -1; j < n; j++) {
        double UL[4], UR[4], Fc[4];
        for (c = 0; c < 4; c++) {
            double tl = or_minmod(AT(Un, c, j) - AT(Un, c, j - 1),
                                  AT(Un, c, j + 1) - AT(Un, c, j)) / h;
            double tr = or_minmod(AT(Un, c, j + 1) - AT(Un, c, j),
                                  AT(Un, c, j + 2) - AT(Un, c, j + 1)) / h;
            double hl = 0.5 * (AT(Un, c, j) + AT(Ut, c, j));
            double hr = 0.5 * (AT(Un, c, j + 1) + AT(Ut, c, j + 1));
            UL[c] = hl + (0.5 * (h - xt[j + G])) * tl;
            UR[c] = hr - (0.5 * (h + xt[j + 1 + G])) * tr;
        }
        cs_flux(g, UL, UR, Fc);
        for (c = 0; c < 4; c++) AT(F, c, j) = Fc[c];
    }

    /* eq. (9) */
    double sumE = 0.0, sumV = 0.0;
    int status = OR_OK;
    for (j = 0; j < n; j++) {
        double Unew[4];
        for (c = 0; c < 4; c++) Unew[c] = AT(Ut, c, j) - dtdx * (AT(F, c, j) - AT(F, c, j - 1));
        U_out[j] = Unew[0];
        U_out[n + j] = Unew[1];
        U_out[2 * n + j] = 0.0;
        U_out[3 * n + j] = Unew[2];
        U_out[4 * n + j] = Unew[3];
        if (xi_out) xi_out[j] = xt[j + G];
        sumE += yE[j + G];
        sumV += yV[j + G];
        double u = Unew[1] / Unew[0];
        double p = (g->gamma - 1.0) * (Unew[2] - 0.5 * Unew[0] * (u * u) - Unew[3]);
        for (c = 0; c < 4; c++)
            if (!isfinite(Unew[c])) status = OR_EPHYS;
        if (!(Unew[0] > 0.0) || !(p > 0.0)) status = OR_EPHYS;
    }
#undef AT
    if (src) {
        src[0] = sumE;
        src[1] = sumV;
    }
    free(Un);
    free(Us);
    free(Ut);
    free(xs);
    free(xt);
    free(un);
    free(F);
    free(yE);
    free(yV);
    return status;
}

/* or_run for the CSPH-TVD step: up to nsteps steps, each with dt from eq.
 * (16) on the current state, stopping at t_end when t_end > *t. */
int cs_run(const or_gas* g, const or_grid* gr, const or_num* nm, double* U, int64_t nsteps,
           double t_end, double* t, int64_t* steps, double* budget, double* dt_last)
{
    int64_t n = gr->nx * gr->ny;
    double* V = (double*)malloc((size_t)(5 * n) * sizeof(double));
    int64_t s;
    int st = OR_OK;
    for (s = 0; s < nsteps; s++) {
        if (t_end > 0.0 && !(*t < t_end)) break;
        double dt = or_dt(g, gr, nm, U);
        if (t_end > 0.0 && *t + dt > t_end) dt = t_end - *t;
        double src[2];
        st = cs_step(g, gr, nm, U, V, *t, dt, src, NULL);
        if (st != OR_OK) break;
        memcpy(U, V, (size_t)(5 * n) * sizeof(double));
        *t += dt;
        *steps += 1;
        if (budget) {
            budget[0] += src[0];
            budget[1] += src[1];
        }
        if (dt_last) *dt_last = dt;
    }
    free(V);
    return st;
}
