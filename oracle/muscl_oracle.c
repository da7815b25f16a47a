/*
 * muscl_oracle.c -- serial FP64 CPU oracle for the Eulerian MUSCL step of
 * Khrapov & Khoperskov, "Dynamics of unstable sound waves in a non-equilibrium
 * medium at the nonlinear stage", J. Phys.: Conf. Ser. 973 (2018) 012007
 * (arXiv:1805.03442).
 *
 * TEST INFRASTRUCTURE. Only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark load this file. The product path (the HIP library) shares
 * no code with it and never calls it.
 *
 * What it computes (one time step of eq. (15), section 2.3):
 *
 *   U^{n+1} = U^n - dt/h (F_{j+1/2} - F_{j-1/2} + G_{k+1/2} - G_{k-1/2}) + dt Y^{n+1/2}
 *
 * for the vibrationally excited gas, eqs. (1)-(5), with U = (rho, rho u, rho v,
 * E, E_nu), closures (6) and the ideal EOS (7).  The pieces, in the order of the
 * step, and the reading taken where the paper is silent:
 *
 *   primitives   W = (rho, u, v, p, E_nu), p from eq. (5), T from eq. (7).
 *   slopes       minmod-limited undivided differences of W (eq. (14) with xi = 0;
 *                the paper does not name its limiter: minmod is our reading).
 *   predictor    primitive (Hancock) half step with the quasi-linear form of
 *                eqs. (1)-(5) and the sources at t^n (section 2.3 names a
 *                two-step predictor-corrector; the predictor's form is our reading).
 *   face states  W^L = W_j^{n+1/2} + sigma_j/2,  W^R = W_{j+1}^{n+1/2} - sigma_{j+1}/2
 *                (eq. (14), xi = 0).
 *   flux         HLL, eq. (13), with the Davis wave speeds printed below it, or
 *                HLLC (Toro's three-wave solver, written here from the
 *                Rankine-Hugoniot conditions across the two outer waves and a
 *                contact with constant normal velocity and pressure).
 *   sources      Y of eq. (15) with the relaxation term in the form of eq. (4)
 *                ((E_nue - E_nu)/tau + rho Q; the printed Y carries an extra rho
 *                factor and a repeated rho f_x -- both read as misprints).
 *   time step    eq. (16) times a CFL number.
 *   boundaries  periodic, reflecting wall or free outflow ends (sections 2.4
 *                and 3), and the forced source of the runs of section 3 at
 *                the x-low end (or_source_ghost), on the whole edge or a
 *                segment of it.
 *   medium      active everywhere, or (2D sector run of section 3) only in a
 *                wedge (or_active).
 *   stiff branch when dt/tau exceeds a threshold, the E_nu equation (4)
 *                (relaxation and pump) is integrated exactly over the (half)
 *                step with E_nue, tau and Q frozen (our addition; the paper's
 *                runs never reach it).
 *
 * Layout: U[c * ncell + k * nx + j], c = 0..4 -> (rho, rho u, rho v, E, E_nu),
 * cell (j, k) centred at ((j + 1/2) h, (k + 1/2) h).  A 1D problem is ny = 1 with
 * rho v = 0: all y work is skipped, which is exactly what the 2D formulas give
 * when every y difference is zero.
 *
 * Every floating-point expression below is written in one explicit order (C
 * evaluates left to right); the build uses -ffp-contract=off so that no
 * multiply-add is fused.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    double gamma, R, Cv;           /* eq. (5), eq. (7); E_nue = rho Cv T       */
    double rho0, T0;               /* reference point of eq. (6)               */
    double tau0, tau_rho, tau_T;   /* tau = tau0 (rho/rho0)^tau_rho (T/T0)^tau_T */
    double Q0, Q_rho, Q_T;         /* Q likewise                               */
    double I0, I_rho, I_T;         /* I likewise                               */
    double fx, fy;                 /* specific external force f, eqs. (2)-(3)  */
} or_gas;

enum { OR_BC_PERIODIC = 0, OR_BC_WALL = 1, OR_BC_OUTFLOW = 2, OR_BC_SOURCE = 3 };
enum { OR_HLLC = 0, OR_HLL = 1 };
enum { OR_OK = 0, OR_EINVAL = -1, OR_EPHYS = -3 };

typedef struct {
    int64_t nx, ny;                /* ny = 1 for 1D                            */
    double h;                      /* cell size                                */
    int32_t bc[4];                 /* x-low, x-high, y-low, y-high             */
    double src_amp;                /* OR_BC_SOURCE (x-low only): density       */
    double src_lambda;             /*   amplitude and wavelength of the wave,  */
    double src_yc, src_hw;         /*   on |y - yc| <= hw (hw <= 0: whole edge) */
    double wedge_x0, wedge_y0;     /* 2D: pump and sink only in the wedge      */
    double wedge_tan;              /*   x >= x0, |y - y0| <= (x - x0) tan      */
} or_grid;                         /*   (wedge_tan <= 0: everywhere)           */

typedef struct {
    double cfl;                    /* multiplies the bound of eq. (16)         */
    int32_t riemann;               /* OR_HLLC or OR_HLL                        */
    double stiff_z;                /* dt/tau threshold of the exact relaxation */
} or_num;

/* ---------------------------------------------------------------- closures */

/* x^a for the power laws of eq. (6).  libm pow in general; for the exponents
 * 0, 1, -1, 2 and 1/2 the correctly rounded IEEE operations 1, x, 1/x, x*x and
 * sqrt(x), i.e. the exact power rounded once. */
static double or_pow(double x, double a)
{
    if (a == 0.0) return 1.0;
    if (a == 1.0) return x;
    if (a == -1.0) return 1.0 / x;
    if (a == 2.0) return x * x;
    if (a == 0.5) return sqrt(x);
    return pow(x, a);
}

/* eq. (6) */
static double or_tau(const or_gas* g, double rho, double T)
{
    return g->tau0 * or_pow(rho / g->rho0, g->tau_rho) * or_pow(T / g->T0, g->tau_T);
}
static double or_Q(const or_gas* g, double rho, double T)
{
    return g->Q0 * or_pow(rho / g->rho0, g->Q_rho) * or_pow(T / g->T0, g->Q_T);
}
static double or_I(const or_gas* g, double rho, double T)
{
    return g->I0 * or_pow(rho / g->rho0, g->I_rho) * or_pow(T / g->T0, g->I_T);
}

/* conserved -> primitive, eq. (5) solved for p */
static void or_prim(const or_gas* g, const double U[5], double W[5])
{
    double gm1 = g->gamma - 1.0;
    double rho = U[0];
    double u = U[1] / rho;
    double v = U[2] / rho;
    double ke = 0.5 * rho * (u * u + v * v);
    W[0] = rho;
    W[1] = u;
    W[2] = v;
    W[3] = gm1 * (U[3] - ke - U[4]);
    W[4] = U[4];
}

/* primitive -> conserved, eq. (5) */
static void or_cons(const or_gas* g, const double W[5], double U[5])
{
    double gm1 = g->gamma - 1.0;
    double rho = W[0], u = W[1], v = W[2], p = W[3], e = W[4];
    U[0] = rho;
    U[1] = rho * u;
    U[2] = rho * v;
    U[3] = p / gm1 + 0.5 * rho * (u * u + v * v) + e;
    U[4] = e;
}

/* minmod of two undivided differences: zero unless both have the same strict
 * sign, else the one of smaller magnitude */
static double or_minmod(double a, double b)
{
    if (a > 0.0 && b > 0.0) return a < b ? a : b;
    if (a < 0.0 && b < 0.0) return a > b ? a : b;
    return 0.0;
}

/* Interface flux along the normal n.  W = (rho, u_n, u_t, p, E_nu); the result
 * F = (mass, normal momentum, tangential momentum, energy, E_nu) fluxes. */
static void or_flux(const or_gas* g, int riemann, const double WL[5], const double WR[5],
                    double F[5])
{
    double gam = g->gamma;
    double gm1 = gam - 1.0;
    double rL = WL[0], uL = WL[1], vL = WL[2], pL = WL[3], eL = WL[4];
    double rR = WR[0], uR = WR[1], vR = WR[2], pR = WR[3], eR = WR[4];

    double EL = pL / gm1 + 0.5 * rL * (uL * uL + vL * vL) + eL;
    double ER = pR / gm1 + 0.5 * rR * (uR * uR + vR * vR) + eR;
    double UL[5] = {rL, rL * uL, rL * vL, EL, eL};
    double UR[5] = {rR, rR * uR, rR * vR, ER, eR};

    /* physical fluxes, the F vector of eq. (15) */
    double mL = rL * uL, mR = rR * uR;
    double FL[5] = {mL, mL * uL + pL, mL * vL, uL * (EL + pL), uL * eL};
    double FR[5] = {mR, mR * uR + pR, mR * vR, uR * (ER + pR), uR * eR};

    /* frozen sound speeds and the wave-speed estimates printed with eq. (13) */
    double cL = sqrt(gam * pL / rL);
    double cR = sqrt(gam * pR / rR);
    double SL = fmin(uL - cL, uR - cR);
    double SR = fmax(uL + cL, uR + cR);

    int c;
    if (riemann == OR_HLL) {
        /* eq. (13) */
        if (0.0 < SL) {
            for (c = 0; c < 5; c++) F[c] = FL[c];
        } else if (SR < 0.0) {
            for (c = 0; c < 5; c++) F[c] = FR[c];
        } else {
            for (c = 0; c < 5; c++)
                F[c] = (SR * FL[c] - SL * FR[c] + SL * SR * (UR[c] - UL[c])) / (SR - SL);
        }
        return;
    }

    /* HLLC: middle wave speed from equal pressure and normal velocity in the two
     * star regions (Rankine-Hugoniot across S_L and S_R). */
    double dL = SL - uL, dR = SR - uR;
    double Ss = (pR - pL + rL * uL * dL - rR * uR * dR) / (rL * dL - rR * dR);

    if (0.0 < SL) {
        for (c = 0; c < 5; c++) F[c] = FL[c];
    } else if (0.0 < Ss) {
        /* left star state: mass, momentum, energy and E_nu jumps across S_L */
        double fac = rL * dL / (SL - Ss);
        double Us[5];
        Us[0] = fac;
        Us[1] = fac * Ss;
        Us[2] = fac * vL;
        Us[3] = fac * (EL / rL + (Ss - uL) * (Ss + pL / (rL * dL)));
        Us[4] = fac * (eL / rL);
        for (c = 0; c < 5; c++) F[c] = FL[c] + SL * (Us[c] - UL[c]);
    } else if (0.0 <= SR) {
        double fac = rR * dR / (SR - Ss);
        double Us[5];
        Us[0] = fac;
        Us[1] = fac * Ss;
        Us[2] = fac * vR;
        Us[3] = fac * (ER / rR + (Ss - uR) * (Ss + pR / (rR * dR)));
        Us[4] = fac * (eR / rR);
        for (c = 0; c < 5; c++) F[c] = FR[c] + SR * (Us[c] - UR[c]);
    } else {
        for (c = 0; c < 5; c++) F[c] = FR[c];
    }
}

/* largest signal speed of eq. (16): max(|v| + c, 2|v|) */
static double or_cell_speed(const or_gas* g, const double U[5])
{
    double W[5];
    or_prim(g, U, W);
    double vel = sqrt(W[1] * W[1] + W[2] * W[2]);
    double c = sqrt(g->gamma * W[3] / W[0]);
    return fmax(vel + c, 2.0 * vel);
}

double or_max_speed(const or_gas* g, const or_grid* gr, const double* U)
{
    int64_t n = gr->nx * gr->ny, i;
    double smax = 0.0;
    for (i = 0; i < n; i++) {
        double Uc[5] = {U[i], U[n + i], U[2 * n + i], U[3 * n + i], U[4 * n + i]};
        double s = or_cell_speed(g, Uc);
        if (s > smax) smax = s;
    }
    return smax;
}

/* eq. (16): dt = cfl * h / max_cells max(|v| + c, 2|v|) */
double or_dt(const or_gas* g, const or_grid* gr, const or_num* nm, const double* U)
{
    return nm->cfl * gr->h / or_max_speed(g, gr, U);
}

/* -------------------------------------------------------------- ghost cells */

/* Map an index outside [0, n) to the cell that fills its ghost, and report
 * whether the normal velocity changes sign there (reflecting wall).  A source
 * end maps like an outflow end; its ghosts are then overwritten by
 * or_source_ghost. */
static int64_t or_ghost(int64_t j, int64_t n, int bc_lo, int bc_hi, int* flip)
{
    *flip = 0;
    if (j >= 0 && j < n) return j;
    int bc = j < 0 ? bc_lo : bc_hi;
    if (bc == OR_BC_PERIODIC) return ((j % n) + n) % n;
    if (bc == OR_BC_OUTFLOW || bc == OR_BC_SOURCE) return j < 0 ? 0 : n - 1;
    /* wall: mirror image */
    *flip = 1;
    return j < 0 ? -1 - j : 2 * n - 1 - j;
}

/*
 * Forced oscillations from a source (section 3, the 1D runs): the ghost
 * cells j = -1, -2 before the x-low end carry a plane sound wave of the
 * frozen sound speed travelling into the domain,
 *
 *   s = a sin(omega t - k x),  k = 2 pi / lambda,  omega = c k,  x = (j + 1/2) h,
 *   rho = rho_b + s,  u = (c / rho_b) s,  v = 0,  p = p_b + c^2 s,
 *   E_nu = E_nu,b + (E_nu,b / rho_b) s,
 *
 * about the steady background at the reference point of eq. (6): rho_b =
 * rho0, p_b = R rho0 T0, E_nu,b = rho0 Cv T0 + rho0 tau0 Q0 (relaxation
 * balancing the pump in eq. (4); without the last term where the ghost lies
 * outside an active wedge, or_active), c = sqrt(gamma p_b / rho_b).  The paper
 * gives the wavelength but neither the amplitude nor the source's form; the
 * frozen-sound plane wave with unchanged specific vibrational energy is our
 * reading.  The E_nu part enters the domain only with the flow's own velocity,
 * i.e. at second order in the amplitude; what pins it is that with frozen
 * relaxation and no pump or sink E_nu / rho stays uniform.  t is the time of
 * the state the step starts from.
 */
static double or_active(const or_grid* gr, int64_t j, int64_t k);

static void or_source_ghost(const or_gas* g, const or_grid* gr, double t, int64_t j, int64_t row,
                            double U[5])
{
    const double pi = 3.141592653589793;
    double rho_b = g->rho0;
    double p_b = g->R * g->rho0 * g->T0;
    double ev_b = g->rho0 * g->Cv * g->T0 + or_active(gr, j, row) * (g->rho0 * g->tau0 * g->Q0);
    double c = sqrt(g->gamma * p_b / rho_b);
    double k = 2.0 * pi / gr->src_lambda;
    double omega = c * k;
    double x = ((double)j + 0.5) * gr->h;
    double s = gr->src_amp * sin(omega * t - k * x);
    double W[5];
    W[0] = rho_b + s;
    W[1] = (c / rho_b) * s;
    W[2] = 0.0;
    W[3] = p_b + (c * c) * s;
    W[4] = ev_b + (ev_b / rho_b) * s;
    or_cons(g, W, U);
}

/*
 * The 2D sector run of section 3: the medium is active (pump Q and sink I of
 * eq. (6)) only inside a wedge with apex (x0, y0) opening towards +x with
 * half-angle atan(wedge_tan); elsewhere Q0 = I0 = 0 and only the relaxation
 * acts.  Evaluated at the centre of cell (j, k), also for ghost cells.  The
 * paper shows the geometry only in a figure; the wedge's placement is our
 * reading.
 */
static double or_active(const or_grid* gr, int64_t j, int64_t k)
{
    if (!(gr->wedge_tan > 0.0)) return 1.0;
    double x = ((double)j + 0.5) * gr->h;
    double y = ((double)k + 0.5) * gr->h;
    double dx = x - gr->wedge_x0;
    return (dx >= 0.0 && fabs(y - gr->wedge_y0) <= dx * gr->wedge_tan) ? 1.0 : 0.0;
}

/* A source end drives the ghosts of row k only on its segment. */
static int or_source_row(const or_grid* gr, int64_t k)
{
    if (!(gr->src_hw > 0.0)) return 1;
    double y = ((double)k + 0.5) * gr->h;
    return fabs(y - gr->src_yc) <= gr->src_hw;
}

/* ------------------------------------------------------------------- step */

typedef struct {
    int64_t nx, ny, nxe, nye, gx, gy; /* extended grid: gx, gy ghosts per side */
} or_ext;

static int64_t ex(const or_ext* e, int64_t j, int64_t k)
{
    return (k + e->gy) * e->nxe + (j + e->gx);
}

/*
 * One MUSCL step, eq. (15), from U_in (the state at time t) to U_out (both
 * ncell*5, may not alias).  dt is given (the caller computes it with or_dt);
 * t matters only to a source end (or_source_ghost).  src[0] receives
 * dt * sum_cells Y_E (the rho (Q - I + v.f) row) and src[1] the summed source
 * increment of E_nu over the step.  Returns OR_OK, or OR_EPHYS if a density or
 * pressure of U_out is not positive or a value is not finite (U_out is then
 * undefined and the caller keeps U_in).
 */
int or_step_at(const or_gas* g, const or_grid* gr, const or_num* nm, const double* U_in,
               double* U_out, double t, double dt, double* src)
{
    const int64_t nx = gr->nx, ny = gr->ny, n = nx * ny;
    const int twod = ny > 1;
    or_ext e;
    e.nx = nx;
    e.ny = ny;
    e.gx = 2;
    e.gy = twod ? 2 : 0;
    e.nxe = nx + 2 * e.gx;
    e.nye = ny + 2 * e.gy;
    const int64_t ne = e.nxe * e.nye;

    const double gam = g->gamma, gm1 = gam - 1.0;
    const double dtdx = dt / gr->h;
    const double hdtdx = 0.5 * dtdx;
    const double hdt = 0.5 * dt;

    double* W = (double*)calloc((size_t)(5 * ne), sizeof(double));   /* W^n       */
    double* Sx = (double*)calloc((size_t)(5 * ne), sizeof(double));  /* sigma_x   */
    double* Sy = (double*)calloc((size_t)(5 * ne), sizeof(double));  /* sigma_y   */
    double* Wh = (double*)calloc((size_t)(5 * ne), sizeof(double));  /* W^{n+1/2} */
    double* Fx = (double*)calloc((size_t)(5 * ne), sizeof(double));  /* F_{j+1/2} */
    double* Gy = (double*)calloc((size_t)(5 * ne), sizeof(double));  /* G_{k+1/2} */
    int64_t j, k;
    int c;

    /* 1. primitives on the extended grid (ghosts filled by the boundary rule;
     *    y-ghost rows first, so x-ghosts of those rows are corners) */
    for (k = -e.gy; k < ny + e.gy; k++) {
        for (j = -e.gx; j < nx + e.gx; j++) {
            int fx_, fy_;
            int64_t js = or_ghost(j, nx, gr->bc[0], gr->bc[1], &fx_);
            int64_t ks = twod ? or_ghost(k, ny, gr->bc[2], gr->bc[3], &fy_) : 0;
            if (!twod) fy_ = 0;
            int64_t s = ks * nx + js;
            double Uc[5] = {U_in[s], U_in[n + s], U_in[2 * n + s], U_in[3 * n + s],
                            U_in[4 * n + s]};
            if (j < 0 && gr->bc[0] == OR_BC_SOURCE && or_source_row(gr, k))
                or_source_ghost(g, gr, t, j, k, Uc);
            if (fx_) Uc[1] = -Uc[1];
            if (fy_) Uc[2] = -Uc[2];
            double Wc[5];
            or_prim(g, Uc, Wc);
            for (c = 0; c < 5; c++) W[c * ne + ex(&e, j, k)] = Wc[c];
        }
    }

    /* 2. limited slopes (eq. (14) with xi = 0) on cells -1..n (one ghost deep) */
    for (k = -(e.gy ? 1 : 0); k < ny + (e.gy ? 1 : 0); k++) {
        for (j = -1; j < nx + 1; j++) {
            int64_t m = ex(&e, j, k);
            for (c = 0; c < 5; c++) {
                const double* q = W + c * ne;
                Sx[c * ne + m] = or_minmod(q[m] - q[m - 1], q[m + 1] - q[m]);
                if (twod)
                    Sy[c * ne + m] = or_minmod(q[m] - q[m - e.nxe], q[m + e.nxe] - q[m]);
            }
        }
    }

    /* 3. predictor: half step of the quasi-linear primitive system with the
     *    sources at t^n.  Rows of A_x sigma_x (normal x) and A_y sigma_y. */
    for (k = -(e.gy ? 1 : 0); k < ny + (e.gy ? 1 : 0); k++) {
        for (j = -1; j < nx + 1; j++) {
            int64_t m = ex(&e, j, k);
            double rho = W[m], u = W[ne + m], v = W[2 * ne + m], p = W[3 * ne + m],
                   ev = W[4 * ne + m];
            double sr = Sx[m], su = Sx[ne + m], sv = Sx[2 * ne + m], sp = Sx[3 * ne + m],
                   se = Sx[4 * ne + m];
            double ax_r = u * sr + rho * su;
            double ax_u = u * su + sp / rho;
            double ax_v = u * sv;
            double ax_p = u * sp + gam * p * su;
            double ax_e = u * se + ev * su;
            double ay_r = 0.0, ay_u = 0.0, ay_v = 0.0, ay_p = 0.0, ay_e = 0.0;
            if (twod) {
                double tr = Sy[m], tu = Sy[ne + m], tv = Sy[2 * ne + m],
                       tp = Sy[3 * ne + m], te = Sy[4 * ne + m];
                ay_r = v * tr + rho * tv;
                ay_u = v * tu;
                ay_v = v * tv + tp / rho;
                ay_p = v * tp + gam * p * tv;
                ay_e = v * te + ev * tv;
            }
            /* sources at t^n: eq. (6), E_nue = rho Cv T, T from eq. (7) */
            double T = p / (g->R * rho);
            double act = or_active(gr, j, k);
            double tau = or_tau(g, rho, T);
            double Q = act * or_Q(g, rho, T);
            double I = act * or_I(g, rho, T);
            double Ee = rho * g->Cv * T;
            /* E_nu gained by relaxation over dt/2 */
            double dEr = hdt * ((Ee - ev) / tau);
            /* stiff: the E_nu equation (4), dE_nu/dt = (E_nue + tau rho Q -
             * E_nu)/tau, solved exactly over dt/2 with E_nue, tau and Q frozen
             * at t^n (relaxation and pump together); the pressure takes the
             * total-energy source rho (Q - I) of eq. (3) less that gain */
            const int stiff = dt / tau > nm->stiff_z;
            double dEv = 0.0;
            if (stiff) dEv = ((Ee + tau * (rho * Q)) - ev) * (-expm1(-(hdt / tau)));
            double r_h, u_h, v_h, p_h, e_h;
            if (twod) {
                r_h = rho - hdtdx * (ax_r + ay_r);
                u_h = u - hdtdx * (ax_u + ay_u) + hdt * g->fx;
                v_h = v - hdtdx * (ax_v + ay_v) + hdt * g->fy;
                if (stiff) {
                    p_h = p - hdtdx * (ax_p + ay_p) - gm1 * (dEv - hdt * (rho * (Q - I)));
                    e_h = ev - hdtdx * (ax_e + ay_e) + dEv;
                } else {
                    p_h = p - hdtdx * (ax_p + ay_p) - gm1 * (dEr + hdt * (rho * I));
                    e_h = ev - hdtdx * (ax_e + ay_e) + (dEr + hdt * (rho * Q));
                }
            } else {
                r_h = rho - hdtdx * ax_r;
                u_h = u - hdtdx * ax_u + hdt * g->fx;
                v_h = v - hdtdx * ax_v + hdt * g->fy;
                if (stiff) {
                    p_h = p - hdtdx * ax_p - gm1 * (dEv - hdt * (rho * (Q - I)));
                    e_h = ev - hdtdx * ax_e + dEv;
                } else {
                    p_h = p - hdtdx * ax_p - gm1 * (dEr + hdt * (rho * I));
                    e_h = ev - hdtdx * ax_e + (dEr + hdt * (rho * Q));
                }
            }
            Wh[m] = r_h;
            Wh[ne + m] = u_h;
            Wh[2 * ne + m] = v_h;
            Wh[3 * ne + m] = p_h;
            Wh[4 * ne + m] = e_h;
        }
    }

    /* 4. x faces j+1/2 for j = -1..nx-1 on interior rows */
    for (k = 0; k < ny; k++) {
        for (j = -1; j < nx; j++) {
            int64_t m = ex(&e, j, k), mr = m + 1;
            double WL[5], WR[5], F[5];
            for (c = 0; c < 5; c++) {
                WL[c] = Wh[c * ne + m] + 0.5 * Sx[c * ne + m];
                WR[c] = Wh[c * ne + mr] - 0.5 * Sx[c * ne + mr];
            }
            or_flux(g, nm->riemann, WL, WR, F);
            for (c = 0; c < 5; c++) Fx[c * ne + m] = F[c];
        }
    }

    /* 5. y faces k+1/2 for k = -1..ny-1 on interior columns; the normal is y,
     *    so the solver sees (rho, v, u, p, E_nu) and returns (., G_v, G_u, ., .) */
    if (twod) {
        for (k = -1; k < ny; k++) {
            for (j = 0; j < nx; j++) {
                int64_t m = ex(&e, j, k), mu = m + e.nxe;
                double WL[5], WR[5], F[5];
                for (c = 0; c < 5; c++) {
                    WL[c] = Wh[c * ne + m] + 0.5 * Sy[c * ne + m];
                    WR[c] = Wh[c * ne + mu] - 0.5 * Sy[c * ne + mu];
                }
                double t;
                t = WL[1]; WL[1] = WL[2]; WL[2] = t;
                t = WR[1]; WR[1] = WR[2]; WR[2] = t;
                or_flux(g, nm->riemann, WL, WR, F);
                t = F[1]; F[1] = F[2]; F[2] = t;
                for (c = 0; c < 5; c++) Gy[c * ne + m] = F[c];
            }
        }
    }

    /* 6-7. sources at t^{n+1/2} and the conservative update, eq. (15) */
    double sumYE = 0.0, sumDe = 0.0;
    int status = OR_OK;
    for (k = 0; k < ny; k++) {
        for (j = 0; j < nx; j++) {
            int64_t m = ex(&e, j, k);
            int64_t s = k * nx + j;
            double rho = Wh[m], u = Wh[ne + m], v = Wh[2 * ne + m], p = Wh[3 * ne + m],
                   ev = Wh[4 * ne + m];
            double T = p / (g->R * rho);
            double act = or_active(gr, j, k);
            double tau = or_tau(g, rho, T);
            double Q = act * or_Q(g, rho, T);
            double I = act * or_I(g, rho, T);
            double Ee = rho * g->Cv * T;
            double Y[5];
            Y[0] = 0.0;
            Y[1] = rho * g->fx;
            Y[2] = rho * g->fy;
            Y[3] = rho * (u * g->fx + v * g->fy + Q - I);
            Y[4] = (Ee - ev) / tau + rho * Q;

            double Un[5], Unew[5];
            for (c = 0; c < 5; c++) Un[c] = U_in[c * n + s];
            for (c = 0; c < 5; c++) {
                double dF = Fx[c * ne + m] - Fx[c * ne + m - 1];
                if (twod) {
                    double dG = Gy[c * ne + m] - Gy[c * ne + m - e.nxe];
                    Unew[c] = Un[c] - dtdx * (dF + dG) + dt * Y[c];
                } else {
                    Unew[c] = Un[c] - dtdx * dF + dt * Y[c];
                }
            }
            double de = dt * Y[4];
            double z = dt / tau;
            if (z > nm->stiff_z) {
                /* the E_nu equation (4) over the whole step, solved exactly
                 * from the start-of-step E_nu with E_nue, tau and Q frozen at
                 * t^{n+1/2}: relaxation toward E_nue + tau rho Q */
                de = ((Ee + tau * (rho * Q)) - Un[4]) * (-expm1(-z));
                if (twod) {
                    double dF = Fx[4 * ne + m] - Fx[4 * ne + m - 1];
                    double dG = Gy[4 * ne + m] - Gy[4 * ne + m - e.nxe];
                    Unew[4] = Un[4] - dtdx * (dF + dG) + de;
                } else {
                    double dF = Fx[4 * ne + m] - Fx[4 * ne + m - 1];
                    Unew[4] = Un[4] - dtdx * dF + de;
                }
            }
            sumYE += dt * Y[3];
            sumDe += de;
            for (c = 0; c < 5; c++) U_out[c * n + s] = Unew[c];

            /* positivity and finiteness (no floors: the step is rejected) */
            double Wn[5];
            or_prim(g, Unew, Wn);
            for (c = 0; c < 5; c++)
                if (!isfinite(Unew[c])) status = OR_EPHYS;
            if (!(Wn[0] > 0.0) || !(Wn[3] > 0.0)) status = OR_EPHYS;
        }
    }
    if (src) {
        src[0] = sumYE;
        src[1] = sumDe;
    }

    free(W);
    free(Sx);
    free(Sy);
    free(Wh);
    free(Fx);
    free(Gy);
    return status;
}

/* or_step_at for boundaries that do not depend on time (t = 0). */
int or_step(const or_gas* g, const or_grid* gr, const or_num* nm, const double* U_in,
            double* U_out, double dt, double* src)
{
    return or_step_at(g, gr, nm, U_in, U_out, 0.0, dt, src);
}

/*
 * Advance U in place by up to nsteps steps, each with dt from eq. (16) on the
 * current state, stopping at t_end (dt is shortened to land on it) when
 * t_end > *t.  On return *t, *steps and budget[2] (running sums of src of
 * or_step) are updated.  Returns OR_OK or the first error (U then holds the last
 * good state).
 */
int or_run(const or_gas* g, const or_grid* gr, const or_num* nm, double* U, int64_t nsteps,
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
        st = or_step_at(g, gr, nm, U, V, *t, dt, src);
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

/* Conversions for the caller (initial data and read-out), eq. (5). */
void or_prim_to_cons(const or_gas* g, int64_t n, const double* W, double* U)
{
    int64_t i;
    int c;
    for (i = 0; i < n; i++) {
        double Wc[5], Uc[5];
        for (c = 0; c < 5; c++) Wc[c] = W[c * n + i];
        or_cons(g, Wc, Uc);
        for (c = 0; c < 5; c++) U[c * n + i] = Uc[c];
    }
}

void or_cons_to_prim(const or_gas* g, int64_t n, const double* U, double* W)
{
    int64_t i;
    int c;
    for (i = 0; i < n; i++) {
        double Wc[5], Uc[5];
        for (c = 0; c < 5; c++) Uc[c] = U[c * n + i];
        or_prim(g, Uc, Wc);
        for (c = 0; c < 5; c++) W[c * n + i] = Wc[c];
    }
}

/* Single interface flux, exposed so that tests can check the Riemann solvers
 * on their own (consistency, contact preservation, upwinding). */
void or_face_flux(const or_gas* g, int32_t riemann, const double* WL, const double* WR,
                  double* F)
{
    or_flux(g, riemann, WL, WR, F);
}

/* Source vector Y of eq. (15) at one primitive state (non-stiff form). */
void or_source(const or_gas* g, const double* W, double* Y)
{
    double rho = W[0], u = W[1], v = W[2], p = W[3], ev = W[4];
    double T = p / (g->R * rho);
    double tau = or_tau(g, rho, T);
    double Q = or_Q(g, rho, T);
    double I = or_I(g, rho, T);
    double Ee = rho * g->Cv * T;
    Y[0] = 0.0;
    Y[1] = rho * g->fx;
    Y[2] = rho * g->fy;
    Y[3] = rho * (u * g->fx + v * g->fy + Q - I);
    Y[4] = (Ee - ev) / tau + rho * Q;
}
