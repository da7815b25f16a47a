// ng_internal.hpp -- data shared by the host side of the library and its HIP
// kernels: per-solve descriptors, mutable per-solve control blocks and the
// per-workgroup reduction records of one step.
//
// Device memory of one solve (inside the caller's buffer):
//   [buffer A: planes x ncell reals][buffer B: same][partials][workgroup table]
// Planes are the conserved components (rho, rho u, [rho v], E, E_nu), each a
// contiguous row-major plane with x fastest (cell (j, k) at k*nx + j).  The FP32
// path stores deviations from a uniform reference state U_ref.
#pragma once

#include <stdint.h>

namespace ng {

constexpr int kWave = 64;          // CDNA wavefront width
constexpr int kHalo = 2;           // ghost cells per side of the stencil
constexpr int kInterior = kWave - 2 * kHalo;  // cells a wave updates per row
constexpr int kMaxWaves = 8;       // waves per workgroup, upper bound

// Schemes of a 1D solve (the values of NG_MUSCL and NG_CSPH_TVD).  A CSPH-TVD
// step reaches three cells to each side (predictor, corrector, face values),
// so its wave segments keep three halo lanes per side.
constexpr int kSchemeMuscl = 0;
constexpr int kSchemeCsph = 1;
constexpr int kCsphHalo = 3;
constexpr int kCsphInterior = kWave - 2 * kCsphHalo;
// cells a wave updates per 1D segment under a scheme
constexpr int seg_cells(int scheme)
{
    return scheme == kSchemeCsph ? kCsphInterior : kInterior;
}

// Boundary kinds of an axis end (the values of NG_BC_*): ghost cells wrap
// around, mirror the interior with the normal momentum negated, or copy the
// edge cell.
constexpr int kBcPeriodic = 0;
constexpr int kBcWall = 1;
constexpr int kBcOutflow = 2;
constexpr int kBcSource = 3;   // x-low only: forced sound wave in the ghosts

// Closure recipes of the FP32 arithmetic: the exponent codes (2a, 2b) of
// 1/tau, Q and I of eq. (6), each written c rho^a p^b with T = p / (R rho),
// compiled into kernels of their own so that the powers are products of rho,
// p, 1/rho and one reciprocal square root instead of two log2 and three exp2.
// The rows are the base gas of eq. (6) (tau ~ 1/(rho T), I ~ rho T^2,
// Q ~ rho^1/2 T^Q_T) with Q_T = 2 and 1; a solve whose codes match a row runs
// that recipe, any other the general form (row 0).
constexpr int kRecipes = 2;
// step kernel variant of a launch whose solves all take the CSPH-TVD step
// (1D, FP64); the closure-recipe variants are 1 .. kRecipes + 1
constexpr int kVariantCsph = kRecipes + 2;
constexpr int kRecipeCodes[kRecipes + 1][6] = {
    {0, 0, 0, 0, 0, 0},
    {0, 2, -3, 4, -2, 4},
    {0, 2, -1, 2, -2, 4},
};

// Run-constant description of one solve.
struct InstDesc {
    int64_t nx, ny, ncell;
    int32_t ndim, riemann;
    int32_t nstrips;          // 2D: column strips of kInterior cells; 1D: segments
                              // of seg_cells(scheme) cells
    int32_t rows_per_item;    // 2D: rows per work item; 1D: segments per work item
    int32_t nchunks;          // 2D: row chunks; 1D: segment groups
    int32_t waves_per_block;
    int32_t fused;            // the step kernel accepts the step (last workgroup)
    int32_t bc[4];            // boundary kinds: x-low, x-high, y-low, y-high
    int32_t any_bc;           // some end is not periodic
    int32_t scheme;           // kSchemeMuscl, or kSchemeCsph (1D, FP64)
    int64_t nitems;           // nstrips * nchunks (2D) or nchunks (1D)
    int64_t nblocks;          // workgroups of this solve's step launch
    uint64_t buf[2];          // device addresses of the two state buffers
    uint64_t partials;        // device address of the per-workgroup records
    // numerics
    double h, cfl, stiff_z;
    // gas, eqs. (5)-(7)
    double gamma, gm1, R, Cv;
    double rho0, T0, tau0, tau_rho, tau_T, Q0, Q_rho, Q_T, I0, I_rho, I_T;
    double fx, fy;
    // reference state of the FP32 deviation storage (zero for FP64)
    double uref[5];           // (rho_r, 0, 0, E_r, Ev_r)
    // the FP32 and mixed states hold E - E_nu (not E) in the energy slot, as a
    // deviation from e1_r = p_r / (gamma - 1); H_r = e1_r + p_r
    double p_r, H_r, D_r, e1_r;   // ..., Cv/R p_r - Ev_r, p_r / (gamma - 1)
    // forced source at the x-low end: s = amp sin(omega t - k x) about the
    // background (rho_b, 0, 0, p_b, E_nu,b); uc = c / rho_b, c2 = c^2,
    // er = E_nu,b / rho_b
    double src_amp, src_k, src_omega;
    double src_rho, src_p, src_ev, src_uc, src_c2, src_er;
    double src_yc, src_hw;    // 2D: the source drives rows with |y - yc| <= hw
    // 2D sector run: pump and sink only for x >= x0, |y - y0| <= (x - x0) tan
    double wedge_x0, wedge_y0, wedge_tan;   // tan <= 0: everywhere
    // The closures of eq. (6) in terms of (rho, p) for the FP32 arithmetic:
    // 1/tau, Q and I = cl_c rho^cl_a p^cl_b (with T = p / (R rho)); cl_recipe
    // > 0 names the compiled recipe whose exponents they are (kRecipeCodes).
    double cl_c[3], cl_a[3], cl_b[3];
    int32_t cl_recipe, pad1;
};

// Mutable per-solve state, advanced by the finalize kernel.
struct InstCtrl {
    double t;                 // time of the state in buf[cur]
    double dt_cfl;            // CFL step of eq. (16) for that state
    double dt_last;           // last step taken
    double t_end;             // stop time (+inf: none)
    int64_t steps;            // steps taken
    int64_t max_steps;        // stop after this many steps
    int32_t cur;              // buffer holding the current state
    int32_t status;           // 0 or NG_EPHYS (sticky)
    uint32_t flags;           // NG_FLAG_* of the current state / last failure
    int32_t reported;         // host bookkeeping for batch polling
    double total[5];          // sum over cells of U (full values, FP64)
    double budget[2];         // sum over steps and cells of the source increments
    double rho_min, p_min, smax;
    uint32_t arrive;          // workgroups of the current step that have finished
    uint32_t pad;
    double src_ghost[3][5];   // forced source: full conserved state of the ghosts
                              // x = -h/2, -3h/2, -5h/2 at time t (set with t;
                              // the third for the CSPH-TVD step's particles)
};

// Grid barrier of a cooperative launch (one solve advanced many steps per
// launch by at most kCoopFlat workgroups that stay resident together), zeroed
// before each launch.  Each step every workgroup writes its signal speed (low
// and high halves) and failure flags into its own slot -- three 8-byte words,
// each (step number << 32 | 32 bits of payload), so that a reader which sees
// the step number in all three words holds one whole message -- and reads
// every slot itself, so that all of them reach the same next dt and
// acceptance.  A workgroup can be at most one step ahead of any other (it
// needs their slots of its current step), so slots by step parity suffice.
constexpr int kCoopFlat = 256;
constexpr int kCoopMaxWaves = 16;   // waves per workgroup of a cooperative launch
struct CoopSync {
    uint32_t stall[32];                // [0]: set by a workgroup whose wait ran out
    uint64_t fslot[2][kCoopFlat][4];   // [step parity][workgroup]
};

// Per-workgroup data of a cooperative launch, in the solve's reduction space:
// records of the workgroup's last two steps (by step parity), written when
// the launch ends, and the workgroup's view of the solve's control when it
// left.
struct CoopRec {
    double tot[5];      // sums of U^{n+1} over the workgroup's cells
    double src[2];      // sums of the source increments of the launch's
                        // accepted steps up to this step, this one included
    double smax, rho_min, p_min;
    uint32_t flags, step;
};
struct CoopView {
    double t, dt_cfl, dt_last;
    int64_t steps, nacc;   // steps of the solve; steps this launch accepted
    int32_t cur, status;
    uint32_t flags, pad;
};
// bytes of reduction space a cooperative launch of G workgroups uses
constexpr uint64_t coop_space(uint64_t G)
{
    return G * (2 * sizeof(CoopRec) + sizeof(CoopView));
}

// Status of a solve whose cooperative launch ended at a wait that ran out of
// polls (the value of NG_ESTALL); like NG_EPHYS it stops the solve, which keeps
// its last accepted step.
constexpr int32_t kStatusStall = -6;

// One workgroup's reduction record of a step (or of the priming pass).
struct Partial {
    double tot[5];
    double src[2];
    double smax, rho_min, p_min;
    uint32_t flags;
    uint32_t pad;
};

// Workgroup -> (solve, local workgroup) map of one batched launch.
struct BlockRef {
    int32_t inst;
    int32_t local;
};

}  // namespace ng
