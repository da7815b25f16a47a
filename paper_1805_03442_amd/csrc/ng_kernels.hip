// ng_kernels.hip -- HIP kernels (gfx950) of one MUSCL step, eq. (15), for
// batches of 1D and 2D periodic solves, plus the per-solve reduction of the
// step's global quantities (dt of eq. (16), FP64 totals and source budgets).
//
// Work decomposition.  A wavefront owns a strip of 64 consecutive x-cells: the
// 60 cells it updates plus 2 halo cells on each side, one cell per lane, so
// every x-neighbour (slopes, face states, fluxes) is one lane away and moves
// through ds_bpermute without LDS allocation or barriers.
//   2D: a work item is (strip, chunk of rows).  The wave marches up the chunk
//       one row per iteration, keeping the rows it still needs (primitive
//       states of three rows, the half-step state and x-slopes of the row being
//       updated, the north face state and the y-flux below it) in registers, so
//       each y-face flux is computed once and each cell is loaded once (plus a
//       2-row halo per chunk).
//   1D: a work item is a group of consecutive 60-cell segments (58 cells and
//       3 halo lanes per side for the CSPH-TVD step of section 2.3, whose
//       particles reach three cells).
// Each cell's arithmetic does not depend on where it sits in a strip or chunk,
// so results are independent of the launch shape.
//
// The step kernel writes U^{n+1} into the other state buffer and, per
// workgroup, the max signal speed of U^{n+1}, the FP64 sums of U^{n+1}, the
// FP64 sums of the source increments, minima of rho and p and failure flags.
// The finalize kernel (one workgroup per solve) folds those records in a fixed
// order, accepts or rejects the step, advances t and computes the next dt.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <math.h>
#include <stdint.h>

#include <mutex>
#include <type_traits>

#include "ng_cell.hpp"
#include "ng_csph.hpp"
#include "ng_internal.hpp"
#include "ng_launch.hpp"

namespace ng {

// ------------------------------------------------------------ cross-lane

// Whole-wavefront DPP shifts: from_left gives lane l the value of lane l-1,
// from_right the value of lane l+1 (the end lanes get 0 through bound_ctrl;
// they are halo lanes whose results are never used).
__device__ __forceinline__ int dpp_l(int v) { return __builtin_amdgcn_mov_dpp(v, 0x138, 0xf, 0xf, true); }
__device__ __forceinline__ int dpp_r(int v) { return __builtin_amdgcn_mov_dpp(v, 0x130, 0xf, 0xf, true); }
__device__ __forceinline__ float from_left(float v) { return __int_as_float(dpp_l(__float_as_int(v))); }
__device__ __forceinline__ float from_right(float v) { return __int_as_float(dpp_r(__float_as_int(v))); }
__device__ __forceinline__ double from_left(double v)
{
    return __hiloint2double(dpp_l(__double2hiint(v)), dpp_l(__double2loint(v)));
}
__device__ __forceinline__ double from_right(double v)
{
    return __hiloint2double(dpp_r(__double2hiint(v)), dpp_r(__double2loint(v)));
}

// face value W + s/2 of a limited linear profile (eq. (14)) as one fused
// multiply-add: the product by 1/2 is exact, so this is the correctly rounded
// W + s/2, the value of the separate multiply and add
__device__ __forceinline__ float face(float w, float s) { return __builtin_fmaf(0.5f, s, w); }
__device__ __forceinline__ double face(double w, double s) { return __builtin_fma(0.5, s, w); }

// keep a value computed here (stops it from being sunk into a later block,
// away from the DPP move it combines with)
__device__ __forceinline__ void pin(float& v) { asm volatile("" : "+v"(v)); }
__device__ __forceinline__ void pin(double& v) { asm volatile("" : "+v"(v)); }

// lane permute through the LDS crossbar (reductions only)
__device__ __forceinline__ double lane_xor(double v, int lane, int m)
{
    const int addr = ((lane ^ m) & 63) << 2;
    int lo = __builtin_amdgcn_ds_bpermute(addr, __double2loint(v));
    int hi = __builtin_amdgcn_ds_bpermute(addr, __double2hiint(v));
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float lane_xor(float v, int lane, int m)
{
    return __int_as_float(__builtin_amdgcn_ds_bpermute(((lane ^ m) & 63) << 2, __float_as_int(v)));
}

// index of a cell coordinate in [-3, n + 62) on a periodic axis of n >= 4
// cells (one wrap suffices when n >= 64; short axes wrap several times)
__device__ __forceinline__ int64_t wrap_axis(int64_t x, int64_t n)
{
    if (x < 0) x += n;
    if (n >= kWave) return x >= n ? x - n : x;
    while (x >= n) x -= n;
    return x;
}

// Cell of coordinate j in [-3, n + 62) on an axis of n >= 4 cells whose ends
// have boundary kinds lo and hi, and whether the normal momentum of the value
// loaded there is to be negated.  Ghosts of a periodic end wrap around, of a
// wall mirror the edge cells (-1 -> 0, -2 -> 1, -3 -> 2), of an outflow end copy the
// edge cell; coordinates beyond the ghost layer (lanes that feed no interior
// cell) are clamped into the axis.
__device__ __forceinline__ int64_t axis_cell(int64_t j, int64_t n, int lo, int hi, bool& flip)
{
    flip = false;
    if (j >= 0 && j < n) return j;
    const int bc = j < 0 ? lo : hi;
    if (bc == kBcPeriodic) return wrap_axis(j, n);
    if (bc == kBcOutflow || bc == kBcSource) return j < 0 ? 0 : n - 1;
    flip = true;
    const int64_t m = j < 0 ? -1 - j : 2 * n - 1 - j;
    return m < 0 ? 0 : (m >= n ? n - 1 : m);
}

// Workgroups are dispatched round-robin over the 8 XCDs; hand each XCD a
// contiguous range of logical workgroups so that neighbouring tiles (which
// share halo rows and columns) meet in the same L2.
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t G)
{
    int64_t x = b & 7, i = b >> 3;
    int64_t q = G >> 3, r = G & 7;
    return (x < r) ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// ------------------------------------------------------------- policies

template <int NC>
struct Plain64 {
    using R = double;
    // the FP64 step needs more than 128 registers; asking for two waves per
    // SIMD trades a few spills for latency hiding (13 % faster at 4096^2)
    static constexpr int kMinWaves = 2;
    // largest workgroup of a cooperative launch (eight waves: two per SIMD)
    static constexpr int kCoopThreads = 512;
    // U^n of the updated row is re-read from cache (no registers to spare)
    static constexpr bool kKeepRows = false;
    // the energy slot holds E itself
    static constexpr bool kSplitE = false;
    // the closure recipes are an FP32 fast path
    static constexpr bool kRecipes = false;
    using St = double;
    using K = K64;
    static __device__ K make(const InstDesc& d, double dt)
    {
        K k;
        k.gam = d.gamma;
        k.gm1 = d.gm1;
        k.R = d.R;
        k.Cv = d.Cv;
        k.rho0 = d.rho0;
        k.T0 = d.T0;
        k.tau0 = d.tau0;
        k.tr = d.tau_rho;
        k.tT = d.tau_T;
        k.Q0 = d.Q0;
        k.Qr = d.Q_rho;
        k.QT = d.Q_T;
        k.I0 = d.I0;
        k.Ir = d.I_rho;
        k.IT = d.I_T;
        k.fx = d.fx;
        k.fy = d.fy;
        k.stiff_z = d.stiff_z;
        k.dt = dt;
        k.dtdx = dt / d.h;
        k.hdtdx = 0.5 * k.dtdx;
        k.hdt = 0.5 * dt;
        k.riemann = d.riemann;
        return k;
    }
    static __device__ void prim(const K& k, const R* U, R* W) { prim64<NC>(k, U, W); }
    static __device__ R speed(const K& k, const R* W) { return speed64<NC>(k, W); }
    template <bool FR = false, int CL = 0>
    static __device__ void predict(const K& k, const R* W, const R* sx, const R* sy, R* Wh,
                                   R act = 1)
    {
        predict64<NC>(k, W, sx, sy, Wh, act);
    }
    template <int RS>
    static __device__ void flux(const K& k, const R* L, const R* Rr, R* F)
    {
        flux64<NC, RS>(k, L, Rr, F);
    }
    template <bool FR = false, int CL = 0>
    static __device__ void update(const K& k, const R* Un, const R* dF, const R* dG, const R* Wh,
                                  R* Unew, R& sE, R& sV, R act = 1)
    {
        update64<NC>(k, Un, dF, dG, Wh, Unew, sE, sV, act);
    }
    static __device__ R full_rho(const K&, R r) { return r; }
    static __device__ R full_p(const K&, R p) { return p; }
};

template <int NC>
struct Dev32 {
    using R = float;
    using St = float;   // stored state: FP32 deviations
    using K = K32;
    static constexpr int kMinWaves = 1;
    // twelve waves (three per SIMD at up to 168 registers, one workgroup per
    // CU): 2^20 cells 12.3 against 13.2 us per step with eight; sixteen-wave
    // workgroups, which force 128 registers, spill and were slower
    static constexpr int kCoopThreads = 768;
    // the raw rows stay in registers until their update
    static constexpr bool kKeepRows = true;
    // the energy slot holds e = E - E_nu (deviation from e_r)
    static constexpr bool kSplitE = true;
    static constexpr bool kRecipes = true;
    static __device__ K make(const InstDesc& d, double dt)
    {
        K k;
        k.gam = (float)d.gamma;
        k.gm1 = (float)d.gm1;
        k.igm1 = (float)(1.0 / d.gm1);
        k.CvR = (float)(d.Cv / d.R);
        k.rho_r = (float)d.uref[0];
        k.p_r = (float)d.p_r;
        k.ev_r = (float)d.uref[4];
        k.H_r = (float)d.H_r;
        k.D_r = (float)d.D_r;
        for (int i = 0; i < 3; i++) {
            k.cl_c[i] = (float)d.cl_c[i];
            k.cl_a[i] = (float)d.cl_a[i];
            k.cl_b[i] = (float)d.cl_b[i];
        }
        k.gp_r = (float)(d.gamma * d.p_r);
        k.fx = (float)d.fx;
        k.fy = (float)d.fy;
        k.stiff_z = (float)d.stiff_z;
        k.hstiff_z = 0.5f * k.stiff_z;
        k.dt = (float)dt;
        k.dtdx = (float)(dt / d.h);
        k.hdtdx = 0.5f * k.dtdx;
        k.hdt = 0.5f * k.dt;
        k.hdtfx = k.hdt * k.fx;
        k.hdtfy = k.hdt * k.fy;
        k.force = d.fx != 0.0 || d.fy != 0.0;
        k.dt64 = (double)k.dt;
        k.hdt64 = (double)k.hdt;
        k.riemann = d.riemann;
        return k;
    }
    static __device__ void prim(const K& k, const R* U, R* W) { prim32<NC>(k, U, W); }
    static __device__ R speed(const K& k, const R* W) { return speed32<NC>(k, W); }
    // FR: the half-step state carries the full density (HLLC faces);
    // CL: closure recipe
    template <bool FR = false, int CL = 0>
    static __device__ void predict(const K& k, const R* W, const R* sx, const R* sy, R* Wh,
                                   R act = 1)
    {
        predict32<NC, FR, CL>(k, W, sx, sy, Wh, act);
    }
    template <int RS>
    static __device__ void flux(const K& k, const R* L, const R* Rr, R* F)
    {
        flux32<NC, RS>(k, L, Rr, F);
    }
    template <bool FR = false, int CL = 0>
    static __device__ void update(const K& k, const R* Un, const R* dF, const R* dG, const R* Wh,
                                  R* Unew, R& sE, R& sV, R act = 1)
    {
        update32<NC, FR, CL>(k, Un, dF, dG, Wh, Unew, sE, sV, act);
    }
    static __device__ R full_rho(const K& k, R r) { return k.rho_r + r; }
    static __device__ R full_p(const K& k, R p) { return k.p_r + p; }
};

// FP32 arithmetic on an FP64 state: the deviations from the reference are
// stored in FP64 and rounded to FP32 where the stencil reads them; the step's
// FP32 increment is added in FP64, so rounding no longer accumulates in the
// stored state (the FP32 store loses ~1e-8 of a perturbation per step).
template <int NC>
struct Mix32 {
    using R = float;
    using St = double;
    using K = K32;
    static constexpr int kMinWaves = 1;
    static constexpr int kCoopThreads = 512;
    static constexpr bool kKeepRows = true;
    static constexpr bool kSplitE = true;
    static constexpr bool kRecipes = true;
    static __device__ K make(const InstDesc& d, double dt) { return Dev32<NC>::make(d, dt); }
    static __device__ void prim(const K& k, const St* U, R* W)
    {
        R D[NC];
        for (int c = 0; c < NC; c++) D[c] = (R)U[c];
        prim32<NC>(k, D, W);
    }
    static __device__ R speed(const K& k, const R* W) { return speed32<NC>(k, W); }
    // FR: the half-step state carries the full density (HLLC faces);
    // CL: closure recipe
    template <bool FR = false, int CL = 0>
    static __device__ void predict(const K& k, const R* W, const R* sx, const R* sy, R* Wh,
                                   R act = 1)
    {
        predict32<NC, FR, CL>(k, W, sx, sy, Wh, act);
    }
    template <int RS>
    static __device__ void flux(const K& k, const R* L, const R* Rr, R* F)
    {
        flux32<NC, RS>(k, L, Rr, F);
    }
    template <bool FR = false, int CL = 0>
    static __device__ void update(const K& k, const St* Un, const R* dF, const R* dG, const R* Wh,
                                  St* Unew, R& sE, R& sV, R act = 1)
    {
        R dU[NC];
        increment32<NC, FR, CL>(k, (R)Un[NC == 5 ? 4 : 3], dF, dG, Wh, dU, sE, sV, act);
        for (int c = 0; c < NC; c++) Unew[c] = Un[c] + (St)dU[c];
    }
    static __device__ R full_rho(const K& k, R r) { return k.rho_r + r; }
    static __device__ R full_p(const K& k, R p) { return k.p_r + p; }
};

// ------------------------------------------------------ reduction records

// Per-lane accumulators of one work item: FP64 sums of the updated conserved
// values and source increments, and the extrema in the working precision.
template <class R>
struct Acc {
    double tot[5];
    double src[2];
    R smax, rmin, pmin;
};

template <class R>
__device__ __forceinline__ void acc_init(Acc<R>& a)
{
    for (int c = 0; c < 5; c++) a.tot[c] = 0.0;
    a.src[0] = a.src[1] = 0.0;
    a.smax = (R)0;
    a.rmin = (R)INFINITY;
    a.pmin = (R)INFINITY;
}

// Record one updated cell: NC conserved values (as stored), its primitives
// and signal speed, and its source increments.  The minima of rho and p are
// kept in the primitives' own form (deviations for FP32) and made full by
// acc_finish: rounding is monotone, so the minimum of the full values is the
// reference plus the minimum deviation.  A split energy slot holds E - E_nu;
// its sum is made the sum of E by acc_finish.
template <class P, int NC>
__device__ __forceinline__ void acc_cell(Acc<typename P::R>& a, const typename P::K& k,
                                         const typename P::St* U, const typename P::R* W,
                                         typename P::R s, typename P::R sE, typename P::R sV)
{
    constexpr int iE = NC == 5 ? 3 : 2, iV = NC - 1;
    a.tot[0] += (double)U[0];
    a.tot[1] += (double)U[1];
    if (NC == 5) a.tot[2] += (double)U[2];
    a.tot[3] += (double)U[iE];
    a.tot[4] += (double)U[iV];
    a.src[0] += (double)sE;
    a.src[1] += (double)sV;
    a.smax = fmax(a.smax, s);
    a.rmin = fmin(a.rmin, W[0]);
    a.pmin = fmin(a.pmin, W[NC == 5 ? 3 : 2]);
}

// Per-lane accumulators as the records expect them: the sum of E (a split
// energy slot summed E - E_nu) and full minima of rho and p.
template <class P>
__device__ __forceinline__ void acc_finish(Acc<typename P::R>& a, const typename P::K& k)
{
    if (P::kSplitE) a.tot[3] += a.tot[4];
    a.rmin = P::full_rho(k, a.rmin);
    a.pmin = P::full_p(k, a.pmin);
}

// Failure flags of a lane: a non-finite value anywhere makes its sums
// non-finite; min/max ignore NaN, so positivity is checked on the extrema.
template <class R>
__device__ __forceinline__ uint32_t acc_flags(const Acc<R>& a)
{
    double all = a.tot[0] + a.tot[1] + a.tot[2] + a.tot[3] + a.tot[4] + a.src[0] + a.src[1];
    uint32_t f = 0u;
    if (!isfinite(all)) f |= 1u;
    if (!(a.rmin > (R)0)) f |= 2u;
    if (!(a.pmin > (R)0)) f |= 4u;
    return f;
}

// Fold the lanes of each wave (lane 0 keeps a fixed-order result), then the
// waves of the workgroup in wave order, and store the workgroup's record
// (WT: with agent-scope stores, which write through to memory).
template <class R, int MaxW = kMaxWaves, bool WT = false>
__device__ __forceinline__ void block_reduce_store(Acc<R>& a, Partial* out, int wave, int lane,
                                                   int nwaves)
{
    __shared__ double sh[MaxW][11];
    __shared__ uint32_t shf[MaxW];
    uint32_t flags = acc_flags(a);
    double smax = (double)a.smax, rmin = (double)a.rmin, pmin = (double)a.pmin;
    for (int m = 32; m >= 1; m >>= 1) {
        for (int c = 0; c < 5; c++) a.tot[c] += lane_xor(a.tot[c], lane, m);
        a.src[0] += lane_xor(a.src[0], lane, m);
        a.src[1] += lane_xor(a.src[1], lane, m);
        smax = fmax(smax, lane_xor(smax, lane, m));
        rmin = fmin(rmin, lane_xor(rmin, lane, m));
        pmin = fmin(pmin, lane_xor(pmin, lane, m));
        flags |= (uint32_t)__builtin_amdgcn_ds_bpermute(((lane ^ m) & 63) << 2, (int)flags);
    }
    if (lane == 0) {
        for (int c = 0; c < 5; c++) sh[wave][c] = a.tot[c];
        sh[wave][5] = a.src[0];
        sh[wave][6] = a.src[1];
        sh[wave][7] = smax;
        sh[wave][8] = rmin;
        sh[wave][9] = pmin;
        shf[wave] = flags;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        Partial r;
        for (int c = 0; c < 5; c++) r.tot[c] = 0.0;
        r.src[0] = r.src[1] = 0.0;
        r.smax = 0.0;
        r.rho_min = INFINITY;
        r.p_min = INFINITY;
        r.flags = 0u;
        r.pad = 0u;
        for (int w = 0; w < nwaves; w++) {
            for (int c = 0; c < 5; c++) r.tot[c] += sh[w][c];
            r.src[0] += sh[w][5];
            r.src[1] += sh[w][6];
            r.smax = fmax(r.smax, sh[w][7]);
            r.rho_min = fmin(r.rho_min, sh[w][8]);
            r.p_min = fmin(r.p_min, sh[w][9]);
            r.flags |= shf[w];
        }
        if constexpr (WT) {
            auto put = [](double* p, double x) {
                __hip_atomic_store(p, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            };
            for (int c = 0; c < 5; c++) put(&out->tot[c], r.tot[c]);
            put(&out->src[0], r.src[0]);
            put(&out->src[1], r.src[1]);
            put(&out->smax, r.smax);
            put(&out->rho_min, r.rho_min);
            put(&out->p_min, r.p_min);
            __hip_atomic_store(&out->flags, r.flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            *out = r;
        }
    }
}

// Control word of a solve as seen by the kernels of one step.
struct StepCtl {
    double dt;
    int cur;
    bool active;
    const double* gsrc;   // forced source: ghost states at the step's start time
};

__device__ __forceinline__ StepCtl read_ctl(const InstCtrl& c)
{
    StepCtl s;
    double t = c.t, t_end = c.t_end;
    s.active = c.status == 0 && t < t_end && c.steps < c.max_steps;
    double dt = c.dt_cfl;
    if (t + dt > t_end) dt = t_end - t;
    s.dt = dt;
    s.cur = c.cur;
    s.gsrc = &c.src_ghost[0][0];
    return s;
}

// A forced-source ghost in the stored form: the full FP64 conserved state
// (5 components; the 1D planes skip rho v) minus the reference (zero in FP64),
// with E - E_nu in the energy slot of a split state.
template <class St, int NC, bool Split>
__device__ __forceinline__ void source_cell(const InstDesc& d, const double* g, St* U)
{
    for (int c = 0; c < NC; c++) {
        const int q = NC == 5 ? c : (c < 2 ? c : c + 1);
        U[c] = (St)(g[q] - d.uref[q]);
    }
    if (Split) U[NC == 5 ? 3 : 2] = (St)((g[3] - g[4]) - d.e1_r);
}

template <class R, int NC>
__device__ __forceinline__ void load_cell(const R* __restrict__ base, int64_t ncell, int64_t idx,
                                          R* U)
{
    for (int c = 0; c < NC; c++) U[c] = base[c * ncell + idx];
}
template <class R, int NC>
__device__ __forceinline__ void load_cell_cached(const R* __restrict__ base, int64_t ncell,
                                                 int64_t idx, R* U)
{
    for (int c = 0; c < NC; c++) U[c] = base[c * ncell + idx];
}

// ==================================================== accepting a step

// Ghost g (cell -1 - g, centre x = -h/2 - g h) of a forced source at the
// x-low end for the time t: the plane sound wave s = a sin(omega t - k x)
// about the background (section 3's forced oscillations), as conserved FP64
// values (eq. (5)).  The step kernels take it from the control block, the
// cooperative kernel computes it itself: the same arithmetic in both.
__device__ __forceinline__ void source_ghost(const InstDesc& d, double t, int g, double* U)
{
    const double x = ((double)(-1 - g) + 0.5) * d.h;
    const double s = d.src_amp * sin(d.src_omega * t - d.src_k * x);
    const double rho = d.src_rho + s;
    const double u = d.src_uc * s;
    const double v = 0.0;
    const double p = d.src_p + d.src_c2 * s;
    const double e = d.src_ev + d.src_er * s;
    U[0] = rho;
    U[1] = rho * u;
    U[2] = rho * v;
    U[3] = p / d.gm1 + 0.5 * rho * (u * u + v * v) + e;
    U[4] = e;
}

// the three ghosts for the time c.t, into the control block
__device__ __noinline__ void source_ghosts(const InstDesc& d, InstCtrl& c)
{
    for (int g = 0; g < 3; g++) source_ghost(d, c.t, g, c.src_ghost[g]);
}
// one ghost, out of line: inlined, the sine's registers would count against
// the cooperative kernel's step loop
__device__ __noinline__ void source_ghost_at(const InstDesc& d, double t, int g, double* U)
{
    source_ghost(d, t, g, U);
}

// Apply a folded step record v = (tot[5], src[2], smax, rho_min, p_min) with
// flags to a solve: reject (sticky NG_EPHYS, buffers not swapped) or accept
// (swap buffers, advance t, next dt from eq. (16)).  mode 1: priming (no step
// taken, only the totals and the first dt).
__device__ void accept_step(const InstDesc& d, InstCtrl& c, const StepCtl& sc, const double* v,
                            uint32_t flags, int mode)
{
    const double n = (double)d.ncell;
    const uint32_t bad = flags & 7u;
    if (bad) {
        c.status = -3;  // NG_EPHYS
        c.flags = bad;
        return;
    }
    if (mode == 0) {
        c.cur = sc.cur ^ 1;
        c.t = c.t + sc.dt;
        c.steps = c.steps + 1;
        c.dt_last = sc.dt;
        c.budget[0] += v[5];
        c.budget[1] += v[6];
    }
    for (int q = 0; q < 5; q++) c.total[q] = v[q] + n * d.uref[q];
    c.smax = v[7];
    c.rho_min = v[8];
    c.p_min = v[9];
    c.dt_cfl = d.cfl * d.h / v[7];
    c.flags = 0u;
    if (d.bc[0] == kBcSource) source_ghosts(d, c);
}

// ================================================================ finalize

// One workgroup per solve: fold the step's records in a fixed order, accept
// (swap buffers, advance t, next dt from eq. (16)) or reject (sticky NG_EPHYS,
// the state before the step is kept).  mode 0: after a step; 1: priming.
// Fold a solve's workgroup records in a fixed order with all threads of the
// calling workgroup (up to 16 waves): strided per-thread sums, then lanes
// (butterfly; lane 0's order is fixed), then waves in order.  The result is in
// out[10] / *oflags, valid in thread 0 after the call.
__device__ void fold_partials(const InstDesc& d, int64_t nb, double* out, uint32_t* oflags)
{
    __shared__ double sh[16][10];
    __shared__ uint32_t shf[16];
    const Partial* parts = (const Partial*)d.partials;
    double tot[5] = {0, 0, 0, 0, 0}, src0 = 0.0, src1 = 0.0, smax = 0.0, rmin = INFINITY,
           pmin = INFINITY;
    uint32_t flags = 0;
#pragma unroll 4
    for (int64_t b = threadIdx.x; b < nb; b += blockDim.x) {
        const Partial& p = parts[b];
        for (int q = 0; q < 5; q++) tot[q] += p.tot[q];
        src0 += p.src[0];
        src1 += p.src[1];
        smax = fmax(smax, p.smax);
        rmin = fmin(rmin, p.rho_min);
        pmin = fmin(pmin, p.p_min);
        flags |= p.flags;
    }
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    for (int m = 32; m >= 1; m >>= 1) {
        for (int q = 0; q < 5; q++) tot[q] += lane_xor(tot[q], lane, m);
        src0 += lane_xor(src0, lane, m);
        src1 += lane_xor(src1, lane, m);
        smax = fmax(smax, lane_xor(smax, lane, m));
        rmin = fmin(rmin, lane_xor(rmin, lane, m));
        pmin = fmin(pmin, lane_xor(pmin, lane, m));
        flags |= (uint32_t)__builtin_amdgcn_ds_bpermute(((lane ^ m) & 63) << 2, (int)flags);
    }
    if (lane == 0) {
        for (int q = 0; q < 5; q++) sh[wave][q] = tot[q];
        sh[wave][5] = src0;
        sh[wave][6] = src1;
        sh[wave][7] = smax;
        sh[wave][8] = rmin;
        sh[wave][9] = pmin;
        shf[wave] = flags;
    }
    __syncthreads();
    if (t == 0) {
        const int nw = blockDim.x >> 6;
        for (int w = 1; w < nw; w++) {
            for (int q = 0; q < 7; q++) sh[0][q] += sh[w][q];
            sh[0][7] = fmax(sh[0][7], sh[w][7]);
            sh[0][8] = fmin(sh[0][8], sh[w][8]);
            sh[0][9] = fmin(sh[0][9], sh[w][9]);
            shf[0] |= shf[w];
        }
        for (int q = 0; q < 10; q++) out[q] = sh[0][q];
        *oflags = shf[0];
    }
}

__global__ void __launch_bounds__(256) finalize_kernel(const InstDesc* __restrict__ descs,
                                                        InstCtrl* __restrict__ ctrls,
                                                        const int32_t* __restrict__ insts,
                                                        int mode)
{
    const int inst = insts[blockIdx.x];
    const InstDesc& d = descs[inst];
    InstCtrl& c = ctrls[inst];
    if (mode == 0 && d.fused) return;   // accepted by the step kernel itself
    const StepCtl sc = read_ctl(c);
    if (mode == 0 && !sc.active) return;
    if (mode == 1 && c.status != 0) return;
    double v[10];
    uint32_t flags;
    fold_partials(d, d.nblocks, v, &flags);
    if (threadIdx.x == 0) accept_step(d, c, sc, v, flags, mode);
}

// The last workgroup of a solve to finish a step folds the solve's records and
// accepts the step, so that a step is a single launch.  Each workgroup
// releases its record (agent-scope release fence) before it counts itself in;
// only the last one acquires (agent-scope acquire fence) before reading all
// records, so the other workgroups never invalidate their caches.  The counter
// is reset by the last one.
__device__ void last_block_accept(const InstDesc& d, InstCtrl& c, const StepCtl& sc)
{
    __shared__ int last;
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const uint32_t prev =
            __hip_atomic_fetch_add(&c.arrive, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        last = prev == (uint32_t)(d.nblocks - 1);
    }
    __syncthreads();
    if (!last) return;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    double v[10];
    uint32_t flags;
    fold_partials(d, d.nblocks, v, &flags);
    if (threadIdx.x == 0) {
        accept_step(d, c, sc, v, flags, 0);
        c.arrive = 0u;
    }
}

// ================================================================ 2D step

// The NC conserved planes of one state buffer: uniform base addresses and a
// 32-bit byte offset per cell (planes are < 4 GiB).  Coh: agent-scope loads
// and stores (the cooperative launch, where the next step's loads must see
// what workgroups on other XCDs stored: the stores write through to memory
// and the loads never take a stale line from this XCD's L2).
typedef __attribute__((address_space(1))) char gchar;

template <class R, int NC, bool Coh = false>
struct Planes {
    typedef __attribute__((address_space(1))) R gR;
    gchar* base[NC];
    __device__ Planes(uint64_t buf, int64_t ncell)
    {
        for (int c = 0; c < NC; c++) base[c] = (gchar*)(buf + (uint64_t)(c * ncell * (int64_t)sizeof(R)));
    }
    __device__ __forceinline__ void load(uint32_t boff, R* U) const
    {
        for (int c = 0; c < NC; c++) {
            if constexpr (Coh)
                U[c] = __hip_atomic_load((gR*)(base[c] + (uint64_t)boff), __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
            else
                U[c] = *(const gR*)(base[c] + (uint64_t)boff);
        }
    }
    __device__ __forceinline__ void store(uint32_t boff, const R* U) const
    {
        for (int c = 0; c < NC; c++) {
            if constexpr (Coh)
                __hip_atomic_store((gR*)(base[c] + (uint64_t)boff), U[c], __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            else
                __builtin_nontemporal_store(U[c], (gR*)(base[c] + (uint64_t)boff));
        }
    }
};

// y-face flux: the normal velocity is v, so the Riemann solver sees
// (rho, v, u, p, E_nu) and returns (., G_v, G_u, ., .)
template <class P, int RS>
__device__ __forceinline__ void flux_y(const typename P::K& k, const typename P::R* N,
                                       const typename P::R* S, typename P::R* G)
{
    using R = typename P::R;
    R a[5] = {N[0], N[2], N[1], N[3], N[4]};
    R b[5] = {S[0], S[2], S[1], S[3], S[4]};
    R f[5];
    P::template flux<RS>(k, a, b, f);
    G[0] = f[0];
    G[1] = f[2];
    G[2] = f[1];
    G[3] = f[3];
    G[4] = f[4];
}

// One work item of the 2D step: strip (60 columns + halo) x chunk of rows.
// CL: closure recipe of the FP32 arithmetic (0: general).
template <class P, int RS, bool BC, int CL = 0>
__device__ __forceinline__ void march2d(const InstDesc& d, const typename P::K& k, int cur,
                                        const double* gsrc, int64_t item, int lane,
                                        Acc<typename P::R>& acc)
{
    using R = typename P::R;
    constexpr int NC = 5;
    // the HLLC flux takes the full density in its face states
    constexpr bool FR = RS == 0;
    const int64_t nx = d.nx, ny = d.ny;
    const int64_t strip = item % d.nstrips, chunk = item / d.nstrips;
    const int64_t x0 = strip * kInterior;
    bool flipx = false;
    const int64_t x = BC ? axis_cell(x0 - kHalo + lane, nx, d.bc[0], d.bc[1], flipx)
                         : wrap_axis(x0 - kHalo + lane, nx);
    const bool inner = lane >= kHalo && lane < kWave - kHalo && x0 + (lane - kHalo) < nx;
    // rows in 32 bits (a grid has fewer than 2^30 cells): the row arithmetic
    // is the same for every lane and stays on the scalar unit
    const int nyi = (int)ny;
    const int r0 = (int)(chunk * d.rows_per_item);
    const int r1 = r0 + d.rows_per_item < nyi ? r0 + d.rows_per_item : nyi;
    using St = typename P::St;
    const Planes<St, NC> src(d.buf[cur], d.ncell);
    const Planes<St, NC> dst(d.buf[cur ^ 1], d.ncell);
    const uint32_t rowb = (uint32_t)(nx * (int64_t)sizeof(St));
    const uint32_t xb = (uint32_t)(x * (int64_t)sizeof(St));
    // byte offset of (row r, this lane's column); r within two rows of [0, ny)
    auto boff = [&](int r) -> uint32_t {
        int rr;
        if (BC) {
            bool f;
            rr = (int)axis_cell(r, ny, d.bc[2], d.bc[3], f);
        } else {
            rr = r < 0 ? r + nyi : (r >= nyi ? r - nyi : r);
        }
        return (uint32_t)rr * rowb + xb;
    };
    // a loaded row r as ghost values: the lanes before a forced source take
    // its wave, wall ghosts carry the mirrored normal momentum (x ends: rho u,
    // y ends: rho v)
    const int64_t xr = x0 - kHalo + lane;
    const bool srcx = BC && d.bc[0] == kBcSource && xr < 0;
    const double* gs = gsrc + (xr == -1 ? 0 : 5);
    // the source drives the ghosts of the rows of its segment (all rows when
    // the segment's half-width is not positive)
    auto src_row = [&](int64_t r) -> bool {
        if (!(d.src_hw > 0.0)) return true;
        const double y = ((double)r + 0.5) * d.h;
        return fabs(y - d.src_yc) <= d.src_hw;
    };
    auto ghost = [&](int64_t r, St* U) {
        if (BC) {
            bool fy;
            (void)axis_cell(r, ny, d.bc[2], d.bc[3], fy);
            if (srcx && src_row(r)) source_cell<St, NC, P::kSplitE>(d, gs, U);
            if (flipx) U[1] = -U[1];
            if (fy) U[2] = -U[2];
        }
    };
    // pump and sink only inside an active wedge (the 2D sector run of section
    // 3): 1 or 0 for this lane's cell centre in row r, ghost cells included
    const bool wedge = BC && d.wedge_tan > 0.0;
    const double xc = ((double)xr + 0.5) * d.h;
    auto active = [&](int64_t r) -> R {
        if (!wedge) return (R)1;
        const double y = ((double)r + 0.5) * d.h;
        const double dx = xc - d.wedge_x0;
        return (dx >= 0.0 && fabs(y - d.wedge_y0) <= dx * d.wedge_tan) ? (R)1 : (R)0;
    };
    auto slopes_x = [&](const R* W, R* sx) {
        for (int c = 0; c < NC; c++) {
            R l = from_left(W[c]), r = from_right(W[c]);
            R a = W[c] - l, b = r - W[c];
            pin(a);
            pin(b);
            sx[c] = minmod(a, b);
        }
    };

    // Rolling state, in two register sets that swap roles every row:
    //   Wd/We  primitive state of rows i+1 / i+2 (and, FP32, 1/rho)
    //   Dp/Dn  y-differences W(i+1) - W(i) / W(i+2) - W(i+1)
    //   h0/h1  half-step state of rows i / i+1;  x0s/x1s their x-slopes
    //   Np/Nn  north face states of rows i / i+1
    //   Gp/Gn  y-fluxes at faces i-1/2 / i+1/2
    //   Uc/Ux  raw row i+2 (arrived) / row i+3 (in flight)
    // Policies that keep the raw rows hold four of them (rows i .. i+3) in a
    // ring U0..U3, so U^n of row i is still in registers at its update;
    // the others re-read it and use U2/U3 only.
    R WA[NC + 1], WB[NC + 1], DA[NC], DB[NC], HA[NC], HB[NC], XA[NC], XB[NC];
    R NA[NC], NB[NC], GA[NC], GB[NC];
    St U0[NC], U1[NC], U2[NC], U3[NC];

    // prologue: rows r0-2 .. r0+1
    {
        R Wa[NC + 1], Wb[NC + 1], Wc[NC + 1], sy[NC], sx[NC], hb[NC], S[NC];
        St t[NC];
        St* t0 = P::kKeepRows ? U0 : t;
        St* t1 = P::kKeepRows ? U1 : t;
        src.load(boff(r0 - 2), t);
        ghost(r0 - 2, t);
        P::prim(k, t, Wa);
        src.load(boff(r0 - 1), t);
        ghost(r0 - 1, t);
        P::prim(k, t, Wb);
        src.load(boff(r0), t0);
        ghost(r0, t0);
        P::prim(k, t0, Wc);
        src.load(boff(r0 + 1), t1);
        ghost(r0 + 1, t1);
        P::prim(k, t1, WA);
        src.load(boff(r0 + 2), U2);
        // row r0-1: its north face state
        slopes_x(Wb, sx);
        for (int c = 0; c < NC; c++) sy[c] = minmod(Wb[c] - Wa[c], Wc[c] - Wb[c]);
        P::template predict<FR, CL>(k, Wb, sx, sy, hb, active(r0 - 1));
        for (int c = 0; c < NC; c++) hb[c] = face(hb[c], sy[c]);
        // row r0
        slopes_x(Wc, XA);
        for (int c = 0; c < NC; c++) {
            R dp = Wc[c] - Wb[c];
            DA[c] = WA[c] - Wc[c];
            sy[c] = minmod(dp, DA[c]);
        }
        P::template predict<FR, CL>(k, Wc, XA, sy, HA, active(r0));
        for (int c = 0; c < NC; c++) {
            S[c] = face(HA[c], -sy[c]);
            NA[c] = face(HA[c], sy[c]);
        }
        flux_y<P, RS>(k, hb, S, GA);
    }

    auto row = [&](int i, R* Wd, R* We, R* Dp, R* Dn, R* h0, R* h1, R* x0s, R* x1s,
                   R* Np, R* Nn, R* Gp, R* Gn, St* Uk, St* Uc, St* Ux) {
        // U^n of row i: kept in the ring (Uk), or else re-read from cache
        // for the update (it was loaded two rows ago).  Loads complete in
        // order, so an FP64 state asks for it before row i+3 and waiting for
        // it does not also wait for the row in flight; an FP32 state asks late
        // and keeps the registers free meanwhile
        constexpr bool reread = !P::kKeepRows;
        constexpr bool early = reread && sizeof(St) == 8;
        St Ul[NC];
        St* Un = reread ? Ul : Uk;
        if (early) src.load(boff(i), Ul);
        // row i+2 has arrived in Uc; put row i+3 in flight.  The load is
        // issued on every row (on the chunk's last row it fetches row i+2
        // again, from cache, into the unused buffer): a load on one path only
        // makes the compiler's wait counts assume the other path, so each row
        // would wait for the loads it has just issued
        ghost(i + 2, Uc);
        P::prim(k, Uc, We);
        src.load(boff(i + 1 < r1 ? i + 3 : i + 2), Ux);
        // predictor of row i+1
        R sy[NC];
        slopes_x(Wd, x1s);
        for (int c = 0; c < NC; c++) {
            Dn[c] = We[c] - Wd[c];
            sy[c] = minmod(Dp[c], Dn[c]);
        }
        P::template predict<FR, CL>(k, Wd, x1s, sy, h1, active(i + 1));
        // y-face i+1/2 between the north state of row i and the south state
        // of row i+1
        {
            R S[NC];
            for (int c = 0; c < NC; c++) {
                S[c] = face(h1[c], -sy[c]);
                Nn[c] = face(h1[c], sy[c]);
            }
            flux_y<P, RS>(k, Np, S, Gn);
        }
        // x-faces of row i: lane j computes face j+1/2 from its east state and
        // lane j+1's west state; face j-1/2 comes from lane j-1
        R dF[NC], dG[NC];
        {
            R E[NC], Wr[NC], Fx[NC];
            for (int c = 0; c < NC; c++) {
                E[c] = face(h0[c], x0s[c]);
                Wr[c] = from_right(face(h0[c], -x0s[c]));
            }
            P::template flux<RS>(k, E, Wr, Fx);
            for (int c = 0; c < NC; c++) {
                dF[c] = Fx[c] - from_left(Fx[c]);
                pin(dF[c]);
                dG[c] = Gn[c] - Gp[c];
            }
        }
        // update of row i
        St Uo[NC];
        R Wn[NC + 1], sE, sV;
        const uint32_t o = boff(i);
        if (reread && !early) src.load(o, Ul);
        P::template update<FR, CL>(k, Un, dF, dG, h0, Uo, sE, sV, active(i));
        P::prim(k, Uo, Wn);
        R s = P::speed(k, Wn);
        if (inner) {
            dst.store(o, Uo);
            acc_cell<P, NC>(acc, k, Uo, Wn, s, sE, sV);
        }
    };

    int i = r0;
    if constexpr (P::kKeepRows) {
        for (; i < r1; i += 4) {
            row(i, WA, WB, DA, DB, HA, HB, XA, XB, NA, NB, GA, GB, U0, U2, U3);
            if (i + 1 >= r1) break;
            row(i + 1, WB, WA, DB, DA, HB, HA, XB, XA, NB, NA, GB, GA, U1, U3, U0);
            if (i + 2 >= r1) break;
            row(i + 2, WA, WB, DA, DB, HA, HB, XA, XB, NA, NB, GA, GB, U2, U0, U1);
            if (i + 3 >= r1) break;
            row(i + 3, WB, WA, DB, DA, HB, HA, XB, XA, NB, NA, GB, GA, U3, U1, U2);
        }
    } else {
        for (; i + 1 < r1; i += 2) {
            row(i, WA, WB, DA, DB, HA, HB, XA, XB, NA, NB, GA, GB, U0, U2, U3);
            row(i + 1, WB, WA, DB, DA, HB, HA, XB, XA, NB, NA, GB, GA, U0, U3, U2);
        }
        if (i < r1) row(i, WA, WB, DA, DB, HA, HB, XA, XB, NA, NB, GA, GB, U0, U2, U3);
    }
}

// periodic solves take the plain wrap-around indexing; solves with a wall or
// outflow end the ghost mapping (a uniform choice per solve)
template <class P, int RS>
__device__ __forceinline__ void march2d_bc(const InstDesc& d, const typename P::K& k, int cur,
                                           const double* gsrc, int64_t item, int lane,
                                           Acc<typename P::R>& acc)
{
    if (d.any_bc)
        march2d<P, RS, true>(d, k, cur, gsrc, item, lane, acc);
    else
        march2d<P, RS, false>(d, k, cur, gsrc, item, lane, acc);
}

// One HLLC work item: a periodic solve whose closures match a compiled recipe
// (kRecipeCodes) takes that recipe's march, every other solve the general
// one.  Every kernel that steps a solve applies this same rule, so a solve's
// state is bitwise the same on every path.
template <class P, int CL = kRecipes>
__device__ __forceinline__ void march2d_hllc(const InstDesc& d, const typename P::K& k, int cur,
                                             const double* gsrc, int64_t item, int lane,
                                             Acc<typename P::R>& acc)
{
    if constexpr (P::kRecipes && CL > 0) {
        if (!d.any_bc && d.cl_recipe == CL) {
            march2d<P, 0, false, CL>(d, k, cur, gsrc, item, lane, acc);
            return;
        }
        march2d_hllc<P, CL - 1>(d, k, cur, gsrc, item, lane, acc);
    } else {
        march2d_bc<P, 0>(d, k, cur, gsrc, item, lane, acc);
    }
}

// V = 0: any solves (boundary kind, flux and closures per solve);
// V = 1 + r: every solve of the launch is periodic with the HLLC flux and its
// closures match recipe r (kRecipeCodes; r = 0: the general form) -- a kernel
// with only that path, and so fewer registers.
template <class P, int V>
__global__ void __launch_bounds__(256, P::kMinWaves) step2d_kernel(const InstDesc* __restrict__ descs,
                                                     InstCtrl* __restrict__ ctrls,
                                                     const BlockRef* __restrict__ blocks,
                                                     int remap, int fused)
{
    using R = typename P::R;
    const int64_t G = gridDim.x;
    const int64_t bid = remap ? xcd_remap(blockIdx.x, G) : (int64_t)blockIdx.x;
    const BlockRef br = blocks[bid];
    const InstDesc& d = descs[br.inst];
    const StepCtl sc = read_ctl(ctrls[br.inst]);
    if (!sc.active) return;
    const typename P::K k = P::make(d, sc.dt);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int nwaves = d.waves_per_block;
    Acc<R> acc;
    acc_init(acc);
    const int64_t item = (int64_t)br.local * nwaves + wave;
    if (item < d.nitems) {
        if constexpr (V > 0)
            march2d<P, 0, false, V - 1>(d, k, sc.cur, sc.gsrc, item, lane, acc);
        else if (d.riemann == 1)
            march2d_bc<P, 1>(d, k, sc.cur, sc.gsrc, item, lane, acc);
        else
            march2d_hllc<P>(d, k, sc.cur, sc.gsrc, item, lane, acc);
    }
    acc_finish<P>(acc, k);
    Partial* parts = (Partial*)d.partials;
    block_reduce_store(acc, parts + br.local, wave, lane, nwaves);
    if (fused && d.fused) last_block_accept(d, ctrls[br.inst], sc);
}

// ================================================================ 1D step

// One work item of the 1D step: a group of consecutive 60-cell segments, or
// with first >= 0 the segments first .. end-1 (the cooperative kernel's share
// of a wave).  The next segment's load is issued before the current one is
// computed.  Coh: agent-scope state loads and stores (Planes).
template <class P, int RS, bool BC, int CL = 0, bool Coh = false>
__device__ __forceinline__ void march1d(const InstDesc& d, const typename P::K& k, int cur,
                                        const double* gsrc, int64_t item, int lane,
                                        Acc<typename P::R>& acc, int64_t first = -1,
                                        int64_t end = -1)
{
    using R = typename P::R;
    constexpr int NC = 4;
    constexpr bool FR = RS == 0;
    const int64_t n = d.nx;
    using St = typename P::St;
    const Planes<St, NC, Coh> src(d.buf[cur], n);
    const Planes<St, NC, Coh> dst(d.buf[cur ^ 1], n);
    const int64_t s0 = first >= 0 ? first : item * d.rows_per_item;
    const int64_t s1 = first >= 0 ? end
                                  : (s0 + d.rows_per_item < d.nstrips ? s0 + d.rows_per_item
                                                                      : d.nstrips);
    auto boff = [&](int64_t sg) -> uint32_t {
        bool f;
        const int64_t x = BC ? axis_cell(sg * kInterior - kHalo + lane, n, d.bc[0], d.bc[1], f)
                             : wrap_axis(sg * kInterior - kHalo + lane, n);
        return (uint32_t)(x * (int64_t)sizeof(St));
    };
    St UA[NC], UB[NC];
    src.load(boff(s0), UA);
    auto seg = [&](int64_t sg, St* Uc, St* Ux) {
        R W[NC + 1], sx[NC], h[NC];
        const uint32_t o = boff(sg);
        // issued on every segment (the last one fetches itself again, from
        // cache, into the unused buffer), so that the compiler's wait counts
        // let the load stay in flight
        src.load(boff(sg + 1 < s1 ? sg + 1 : sg), Ux);
        if (BC) {
            // the lanes before a forced source take its wave; wall ghosts
            // carry the mirrored momentum
            bool f;
            const int64_t xr = sg * kInterior - kHalo + lane;
            (void)axis_cell(xr, n, d.bc[0], d.bc[1], f);
            if (d.bc[0] == kBcSource && xr < 0) source_cell<St, NC, P::kSplitE>(d, gsrc + (xr == -1 ? 0 : 5), Uc);
            if (f) Uc[1] = -Uc[1];
        }
        P::prim(k, Uc, W);
        for (int c = 0; c < NC; c++) {
            R l = from_left(W[c]), r = from_right(W[c]);
            R a = W[c] - l, b = r - W[c];
            pin(a);
            pin(b);
            sx[c] = minmod(a, b);
        }
        P::template predict<FR, CL>(k, W, sx, sx, h);
        R E[NC], Wr[NC], Fx[NC], dF[NC];
        for (int c = 0; c < NC; c++) {
            E[c] = face(h[c], sx[c]);
            Wr[c] = from_right(face(h[c], -sx[c]));
        }
        P::template flux<RS>(k, E, Wr, Fx);
        for (int c = 0; c < NC; c++) {
            dF[c] = Fx[c] - from_left(Fx[c]);
            pin(dF[c]);
        }
        St Uo[NC];
        R Wn[NC + 1], sE, sV;
        P::template update<FR, CL>(k, Uc, dF, dF, h, Uo, sE, sV);
        P::prim(k, Uo, Wn);
        R s = P::speed(k, Wn);
        const bool inner =
            lane >= kHalo && lane < kWave - kHalo && sg * kInterior + (lane - kHalo) < n;
        if (inner) {
            dst.store(o, Uo);
            acc_cell<P, NC>(acc, k, Uo, Wn, s, sE, sV);
        }
    };
    int64_t sg = s0;
    for (; sg + 1 < s1; sg += 2) {
        seg(sg, UA, UB);
        seg(sg + 1, UB, UA);
    }
    if (sg < s1) seg(sg, UA, UB);
}

template <class P, int RS, bool Coh = false>
__device__ __forceinline__ void march1d_bc(const InstDesc& d, const typename P::K& k, int cur,
                                           const double* gsrc,
                                           int64_t item, int lane, Acc<typename P::R>& acc,
                                           int64_t first = -1, int64_t end = -1)
{
    if (d.any_bc)
        march1d<P, RS, true, 0, Coh>(d, k, cur, gsrc, item, lane, acc, first, end);
    else
        march1d<P, RS, false, 0, Coh>(d, k, cur, gsrc, item, lane, acc, first, end);
}

// the 1D counterpart of march2d_hllc
template <class P, int CL = kRecipes, bool Coh = false>
__device__ __forceinline__ void march1d_hllc(const InstDesc& d, const typename P::K& k, int cur,
                                             const double* gsrc, int64_t item, int lane,
                                             Acc<typename P::R>& acc, int64_t first = -1,
                                             int64_t end = -1)
{
    if constexpr (P::kRecipes && CL > 0) {
        if (!d.any_bc && d.cl_recipe == CL) {
            march1d<P, 0, false, CL, Coh>(d, k, cur, gsrc, item, lane, acc, first, end);
            return;
        }
        march1d_hllc<P, CL - 1, Coh>(d, k, cur, gsrc, item, lane, acc, first, end);
    } else {
        march1d_bc<P, 0, Coh>(d, k, cur, gsrc, item, lane, acc, first, end);
    }
}

// CSPH-TVD step (section 2.3) of the segments of work item `item`: lane l of
// a segment holds the particle of cell sg * 58 - 3 + l (ghost particles by the
// boundary rule, a wall ghost with its momentum negated, the three before a
// forced source with its wave at the step's start time, gsrc).  Neighbours are one
// lane away, so each stage is one DPP shift per quantity:
//   predictor (eq. (10)) on lanes 1..62: U* = U^n + dt Y(U^n), xi* = dt (u^n +
//     u*)/2, with every particle at its cell centre;
//   corrector (eq. (11)) on lanes 2..61: U~ = (U^n + U*)/2 + dt/2 Y(U*, xi*),
//     xi~ = xi*/2 + dt/2 (u^n + u~)/2;
//   face j+1/2 on lanes 2..60: HLL (eq. (13)) between U^L = U^{n+1/2}_j +
//     (h - xi~_j) Theta_j / 2 and U^R = U^{n+1/2}_{j+1} - (h + xi~_{j+1})
//     Theta_{j+1} / 2 (eq. (14)), U^{n+1/2} = (U^n + U~)/2;
//   update (eq. (9)) on lanes 3..60: U^{n+1} = U~ - dt/h (F_{j+1/2} - F_{j-1/2}).
// FP64 only (the state is stored whole).  With first >= 0 the segments first
// .. end-1 (the cooperative kernel's share of a wave); Coh: agent-scope state
// loads and stores (Planes).
template <class P, bool BC, bool Coh = false>
__device__ __forceinline__ void march_csph(const InstDesc& d, const K64& k, int cur,
                                           const double* gsrc, int64_t item, int lane,
                                           Acc<double>& acc, int64_t first = -1,
                                           int64_t end = -1)
{
    static_assert(std::is_same<typename P::K, K64>::value, "CSPH-TVD runs on the FP64 state");
    constexpr int NC = 4;
    const int64_t n = d.nx;
    const Planes<double, NC, Coh> src(d.buf[cur], n);
    const Planes<double, NC, Coh> dst(d.buf[cur ^ 1], n);
    const int64_t s0 = first >= 0 ? first : item * d.rows_per_item;
    const int64_t s1 = first >= 0 ? end
                                  : (s0 + d.rows_per_item < d.nstrips ? s0 + d.rows_per_item
                                                                      : d.nstrips);
    const double h = d.h, wn = 2.0 / (3.0 * (h * h));
    // the predictor's particles sit at the centres: distances +-h exactly
    const double g1 = csph_grad_w(h, h, wn), g2 = csph_grad_w(-h, h, wn);
    const double dt = k.dt, hdt = k.hdt, dtdx = k.dtdx;
    auto coord = [&](int64_t sg) { return sg * kCsphInterior - kCsphHalo + lane; };
    auto boff = [&](int64_t sg) -> uint32_t {
        bool f;
        const int64_t x = BC ? axis_cell(coord(sg), n, d.bc[0], d.bc[1], f) : wrap_axis(coord(sg), n);
        return (uint32_t)(x * (int64_t)sizeof(double));
    };
    double UA[NC], UB[NC];
    src.load(boff(s0), UA);
    auto seg = [&](int64_t sg, double* Un, double* Ux) {
        const uint32_t o = boff(sg);
        src.load(boff(sg + 1 < s1 ? sg + 1 : sg), Ux);
        if (BC) {
            bool f;
            const int64_t xr = coord(sg);
            (void)axis_cell(xr, n, d.bc[0], d.bc[1], f);
            if (d.bc[0] == kBcSource && xr < 0 && xr >= -kCsphHalo)
                source_cell<double, NC, false>(d, gsrc + 5 * (-1 - xr), Un);
            if (f) Un[1] = -Un[1];
        }
        // predictor
        double un, pn, phin;
        csph_prim(k, Un, un, pn, phin);
        double Y[NC], sEp, sVp, sEc, sVc;
        csph_y(k, h, g1, g2, from_left(phin), from_left(un), from_right(phin), from_right(un),
               Un[0], un, pn, Un[3], phin, Y, sEp, sVp);
        double Us[NC];
        for (int c = 0; c < NC; c++) Us[c] = Un[c] + dt * Y[c];
        double us, ps, phis;
        csph_prim(k, Us, us, ps, phis);
        const double xs = dt * (0.5 * (un + us));
        // corrector, at the predicted positions
        const double ga = csph_grad_w(h + (xs - from_left(xs)), h, wn);
        const double gb = csph_grad_w(-h + (xs - from_right(xs)), h, wn);
        csph_y(k, h, ga, gb, from_left(phis), from_left(us), from_right(phis), from_right(us),
               Us[0], us, ps, Us[3], phis, Y, sEc, sVc);
        double Ut[NC];
        for (int c = 0; c < NC; c++) Ut[c] = 0.5 * (Un[c] + Us[c]) + hdt * Y[c];
        const double ut = Ut[1] / Ut[0];
        const double xt = 0.5 * xs + hdt * (0.5 * (un + ut));
        // face j+1/2: this particle's profile gives U^L, the right neighbour's U^R
        const double al = 0.5 * (h - xt), ar = 0.5 * (h + xt);
        double UL[NC], UR[NC], F[NC];
        for (int c = 0; c < NC; c++) {
            const double l = from_left(Un[c]), r = from_right(Un[c]);
            double a = Un[c] - l, b = r - Un[c];
            pin(a);
            pin(b);
            const double th = minmod(a, b) / h;
            const double hl = 0.5 * (Un[c] + Ut[c]);
            UL[c] = hl + al * th;
            UR[c] = from_right(hl - ar * th);
        }
        csph_flux(k, UL, UR, F);
        double Uo[NC], Wn[NC];
        for (int c = 0; c < NC; c++) {
            double dF = F[c] - from_left(F[c]);
            pin(dF);
            Uo[c] = Ut[c] - dtdx * dF;
        }
        prim64<NC>(k, Uo, Wn);
        const double s = speed64<NC>(k, Wn);
        const bool inner = lane >= kCsphHalo && lane < kWave - kCsphHalo &&
                           sg * kCsphInterior + (lane - kCsphHalo) < n;
        if (inner) {
            dst.store(o, Uo);
            acc_cell<P, NC>(acc, k, Uo, Wn, s, hdt * sEp + hdt * sEc, hdt * sVp + hdt * sVc);
        }
    };
    int64_t sg = s0;
    for (; sg + 1 < s1; sg += 2) {
        seg(sg, UA, UB);
        seg(sg + 1, UB, UA);
    }
    if (sg < s1) seg(sg, UA, UB);
}

// the FP64 1D step of a solve under its scheme (the MUSCL step on the other
// arithmetic)
template <class P>
__device__ __forceinline__ void march1d_any(const InstDesc& d, const typename P::K& k, int cur,
                                            const double* gsrc, int64_t item, int lane,
                                            Acc<typename P::R>& acc)
{
    if constexpr (std::is_same<typename P::K, K64>::value) {
        if (d.scheme == kSchemeCsph) {
            if (d.any_bc)
                march_csph<P, true>(d, k, cur, gsrc, item, lane, acc);
            else
                march_csph<P, false>(d, k, cur, gsrc, item, lane, acc);
            return;
        }
    }
    if (d.riemann == 1)
        march1d_bc<P, 1>(d, k, cur, gsrc, item, lane, acc);
    else
        march1d_hllc<P>(d, k, cur, gsrc, item, lane, acc);
}

// V as for step2d_kernel, or kVariantCsph: every solve of the launch takes the
// CSPH-TVD step (a kernel with that path only)
template <class P, int V>
__global__ void __launch_bounds__(256) step1d_kernel(const InstDesc* __restrict__ descs,
                                                     InstCtrl* __restrict__ ctrls,
                                                     const BlockRef* __restrict__ blocks,
                                                     int remap, int fused)
{
    using R = typename P::R;
    const int64_t G = gridDim.x;
    const int64_t bid = remap ? xcd_remap(blockIdx.x, G) : (int64_t)blockIdx.x;
    const BlockRef br = blocks[bid];
    const InstDesc& d = descs[br.inst];
    const StepCtl sc = read_ctl(ctrls[br.inst]);
    if (!sc.active) return;
    const typename P::K k = P::make(d, sc.dt);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int nwaves = d.waves_per_block;
    Acc<R> acc;
    acc_init(acc);
    const int64_t item = (int64_t)br.local * nwaves + wave;
    if (item < d.nitems) {
        if constexpr (V == kVariantCsph) {
            if (d.any_bc)
                march_csph<P, true>(d, k, sc.cur, sc.gsrc, item, lane, acc);
            else
                march_csph<P, false>(d, k, sc.cur, sc.gsrc, item, lane, acc);
        } else if constexpr (V > 0) {
            march1d<P, 0, false, V - 1>(d, k, sc.cur, sc.gsrc, item, lane, acc);
        } else {
            march1d_any<P>(d, k, sc.cur, sc.gsrc, item, lane, acc);
        }
    }
    acc_finish<P>(acc, k);
    Partial* parts = (Partial*)d.partials;
    block_reduce_store(acc, parts + br.local, wave, lane, nwaves);
    if (fused && d.fused) last_block_accept(d, ctrls[br.inst], sc);
}

// ============================================================ priming pass

// Signal speed, sums and checks of the current state (no step): the records
// from which the finalize kernel derives the first dt and the totals.
template <class P, int NC>
__global__ void __launch_bounds__(256) prime_kernel(const InstDesc* __restrict__ descs,
                                                    InstCtrl* __restrict__ ctrls,
                                                    const BlockRef* __restrict__ blocks, int inst)
{
    using R = typename P::R;
    // without a workgroup table the launch covers the workgroups of one solve
    const BlockRef br = blocks ? blocks[blockIdx.x] : BlockRef{inst, (int32_t)blockIdx.x};
    const InstDesc& d = descs[br.inst];
    const InstCtrl& cc = ctrls[br.inst];
    if (cc.status != 0) return;
    const typename P::K k = P::make(d, 0.0);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int nwaves = d.waves_per_block;
    Acc<R> acc;
    acc_init(acc);
    const int64_t item = (int64_t)br.local * nwaves + wave;
    if (item < d.nitems) {
        using St = typename P::St;
        const St* __restrict__ src = (const St*)d.buf[cc.cur];
        const int64_t nx = d.nx, ncell = d.ncell;
        int64_t xs, rows0, rows1, seg0, seg1;
        if (NC == 5) {
            const int64_t strip = item % d.nstrips, chunk = item / d.nstrips;
            xs = strip * kInterior;
            rows0 = chunk * d.rows_per_item;
            rows1 = rows0 + d.rows_per_item < d.ny ? rows0 + d.rows_per_item : d.ny;
            seg0 = 0;
            seg1 = 1;
        } else {
            xs = 0;
            rows0 = 0;
            rows1 = 1;
            seg0 = item * d.rows_per_item;
            seg1 = seg0 + d.rows_per_item < d.nstrips ? seg0 + d.rows_per_item : d.nstrips;
        }
        const int w = NC == 5 ? kInterior : seg_cells(d.scheme);
        for (int64_t sg = seg0; sg < seg1; sg++) {
            const int64_t xbase = NC == 5 ? xs : sg * w;
            const int64_t xo = xbase + (lane - kHalo);
            const bool inner = lane >= kHalo && lane < kHalo + w && xo < nx;
            if (!inner) continue;
            for (int64_t r = rows0; r < rows1; r++) {
                St U[NC];
                R W[NC + 1];
                load_cell_cached<St, NC>(src, ncell, r * nx + xo, U);
                P::prim(k, U, W);
                R s = P::speed(k, W);
                acc_cell<P, NC>(acc, k, U, W, s, (R)0, (R)0);
            }
        }
    }
    acc_finish<P>(acc, k);
    Partial* parts = (Partial*)d.partials;
    block_reduce_store(acc, parts + br.local, wave, lane, nwaves);
}

// Set the stop condition of a set of solves (a kernel, so that it can sit in
// the stream between captured graphs without a host copy).
__global__ void set_limits_kernel(InstCtrl* __restrict__ ctrls, const int32_t* __restrict__ insts,
                                  int n, double t_end, int64_t max_steps_from_now)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    InstCtrl& c = ctrls[insts[i]];
    c.t_end = t_end;
    c.max_steps = max_steps_from_now < 0 ? INT64_MAX : c.steps + max_steps_from_now;
}

// ====================================================== small solves

// One workgroup advances one small solve through up to nsteps steps without
// returning to the host: its waves share the solve's work items, fold their
// records through LDS in wave order, and wave 0 accepts the step before the
// next one starts.  Per-cell arithmetic is that of the step kernels, so the
// state is bitwise the same as with one launch per step.
template <class P, int NC>
__global__ void __launch_bounds__(512) run_small_kernel(const InstDesc* __restrict__ descs,
                                                        InstCtrl* __restrict__ ctrls,
                                                        const int32_t* __restrict__ insts,
                                                        int64_t nsteps)
{
    using R = typename P::R;
    const int inst = insts[blockIdx.x];
    const InstDesc& d = descs[inst];
    InstCtrl& c = ctrls[inst];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int nw = blockDim.x >> 6;
    __shared__ double sh[kMaxWaves][10];
    __shared__ uint32_t shf[kMaxWaves];
    for (int64_t st = 0; st < nsteps; st++) {
        const StepCtl sc = read_ctl(c);
        if (!sc.active) break;
        const typename P::K k = P::make(d, sc.dt);
        Acc<R> acc;
        acc_init(acc);
        for (int64_t item = wave; item < d.nitems; item += nw) {
            if constexpr (NC == 5) {
                if (d.riemann == 1)
                    march2d_bc<P, 1>(d, k, sc.cur, sc.gsrc, item, lane, acc);
                else
                    march2d_hllc<P>(d, k, sc.cur, sc.gsrc, item, lane, acc);
            } else {
                march1d_any<P>(d, k, sc.cur, sc.gsrc, item, lane, acc);
            }
        }
        acc_finish<P>(acc, k);
        uint32_t flags = acc_flags(acc);
        double smax = (double)acc.smax, rmin = (double)acc.rmin, pmin = (double)acc.pmin;
        for (int m = 32; m >= 1; m >>= 1) {
            for (int q = 0; q < 5; q++) acc.tot[q] += lane_xor(acc.tot[q], lane, m);
            acc.src[0] += lane_xor(acc.src[0], lane, m);
            acc.src[1] += lane_xor(acc.src[1], lane, m);
            smax = fmax(smax, lane_xor(smax, lane, m));
            rmin = fmin(rmin, lane_xor(rmin, lane, m));
            pmin = fmin(pmin, lane_xor(pmin, lane, m));
            flags |= (uint32_t)__builtin_amdgcn_ds_bpermute(((lane ^ m) & 63) << 2, (int)flags);
        }
        if (lane == 0) {
            for (int q = 0; q < 5; q++) sh[wave][q] = acc.tot[q];
            sh[wave][5] = acc.src[0];
            sh[wave][6] = acc.src[1];
            sh[wave][7] = smax;
            sh[wave][8] = rmin;
            sh[wave][9] = pmin;
            shf[wave] = flags;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int w = 1; w < nw; w++) {
                for (int q = 0; q < 7; q++) sh[0][q] += sh[w][q];
                sh[0][7] = fmax(sh[0][7], sh[w][7]);
                sh[0][8] = fmin(sh[0][8], sh[w][8]);
                sh[0][9] = fmin(sh[0][9], sh[w][9]);
                shf[0] |= shf[w];
            }
            accept_step(d, c, sc, sh[0], shf[0], 0);
        }
        __syncthreads();
    }
}

// ================================================== cooperative solves

// this wave's memory operations have completed: vmcnt(0) lgkmcnt(0) (flat
// stores count in both)
__device__ __forceinline__ void wait_mem() { __builtin_amdgcn_s_waitcnt(0x0070); }

// One 1D solve advanced through up to nsteps steps by one cooperative launch
// of G workgroups that stay resident together (no launch per step).  Every
// workgroup tracks the solve's control (t, steps, buffer, CFL step) itself,
// alike.  Each step its waves march their segments (wave g of the W in the
// launch takes the run [g S / W, (g + 1) S / W) of the S segments: equal
// counts to within one, neighbours' halos in the same cache lines) with
// agent-scope state loads and stores (the stores write through to memory and
// the loads never take a stale line of its own XCD's L2); each workgroup
// reduces its signal speed and failure flags, writes them to its slot of the
// CoopSync block, and reads all G slots: every workgroup then decides the
// step alike (eq. (16)'s next CFL step, or rejection).  The FP64 sums of the
// steps (totals, source budgets, extrema) never cross the barrier: each lane
// keeps those of its last computed and last accepted step, each workgroup
// folds them into its records when the launch ends, and a kernel after the
// launch (coop_after_kernel) folds the records of the last accepted step into
// the control block.  Per-
// cell arithmetic, t and dt follow the step kernels and the finalize kernel
// operation for operation, so the state, t and dt are bitwise those of one
// launch per step; only the summation order of the FP64 totals differs.
// Every wait is bounded by spin_limit polls: a workgroup whose wait runs out
// sets the stall word and leaves, the others leave when their own next wait
// runs out, and the solve keeps the last step a barrier accepted.  A forced
// source's ghosts follow t: every workgroup computes them for its own t (the
// same arithmetic as the control block's), and the after-kernel leaves the
// control block's for the last accepted step.

// Wave-wide wait of a cooperative launch of G <= kCoopFlat workgroups for
// every workgroup's (step << 32 | payload) words of step gen: lane j reads
// slot j (and slot j + 64 when Two), at most spin_limit polls after the first.
// On return m and f hold the largest signal speed and the union of the flags
// of this lane's slots; true when the wait ran out.
static_assert(kCoopFlat <= 4 * kWave, "the slot waits read at most four slots per lane");

// The same wait for 128 < G <= 256 workgroups: lane j reads slots j, j + 64,
// j + 128, j + 192; a slot seen whole is folded at once (max and or are
// idempotent, so a slot folded in an earlier poll may be folded again).  Out
// of line: inlined, its twelve loads in flight cost the step loop registers.
__device__ __noinline__ bool poll_slots4(const uint64_t (*slot)[4], uint32_t G, uint32_t gen,
                                            int lane, int32_t spin_limit, double& m, uint32_t& f)
{
    m = 0.0;
    f = 0u;
    for (int32_t n = 0;; n++) {
        bool have = true;
        uint64_t w[4][3];
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const uint32_t j = (uint32_t)lane + 64u * (uint32_t)q;
            const uint64_t* sl = slot[j < G ? j : 0];
#pragma unroll
            for (int x = 0; x < 3; x++)
                w[q][x] = j < G ? __hip_atomic_load(sl + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                : ((uint64_t)gen << 32);
        }
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const uint32_t j = (uint32_t)lane + 64u * (uint32_t)q;
            if ((uint32_t)(w[q][0] >> 32) == gen && (uint32_t)(w[q][1] >> 32) == gen &&
                (uint32_t)(w[q][2] >> 32) == gen) {
                if (j < G) {
                    m = fmax(m, __longlong_as_double(
                                    (long long)((w[q][0] & 0xffffffffull) | (w[q][1] << 32))));
                    f |= (uint32_t)w[q][2];
                }
            } else {
                have = false;
            }
        }
        if (__builtin_amdgcn_ballot_w64(!have) == 0ull) return false;
        if (n >= spin_limit) return true;
        __builtin_amdgcn_s_sleep(2);
    }
}
template <bool Two>
__device__ __forceinline__ bool poll_slots(const uint64_t (*slot)[4], uint32_t G, uint32_t gen,
                                           int lane, int32_t spin_limit, double& m, uint32_t& f)
{
    const bool mine = (uint32_t)lane < G, mine2 = Two && (uint32_t)lane + 64u < G;
    const uint64_t* sl = slot[mine ? lane : 0];
    const uint64_t* sl2 = slot[mine2 ? lane + 64 : 0];
    uint64_t w0 = 0, w1 = 0, w2 = 0, x0 = 0, x1 = 0, x2 = 0;
    bool stalled = false;
    for (int32_t n = 0;; n++) {
        if (mine) {
            w0 = __hip_atomic_load(sl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            w1 = __hip_atomic_load(sl + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            w2 = __hip_atomic_load(sl + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (Two && mine2) {
            x0 = __hip_atomic_load(sl2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            x1 = __hip_atomic_load(sl2 + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            x2 = __hip_atomic_load(sl2 + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        bool have = !mine || ((uint32_t)(w0 >> 32) == gen && (uint32_t)(w1 >> 32) == gen &&
                              (uint32_t)(w2 >> 32) == gen);
        if (Two)
            have = have && (!mine2 || ((uint32_t)(x0 >> 32) == gen &&
                                       (uint32_t)(x1 >> 32) == gen &&
                                       (uint32_t)(x2 >> 32) == gen));
        if (__builtin_amdgcn_ballot_w64(!have) == 0ull) break;
        if (n >= spin_limit) {
            stalled = true;
            break;
        }
        __builtin_amdgcn_s_sleep(2);
    }
    m = mine ? __longlong_as_double((long long)((w0 & 0xffffffffull) | (w1 << 32))) : 0.0;
    f = mine ? (uint32_t)w2 : 0u;
    if (Two && mine2) {
        m = fmax(m, __longlong_as_double((long long)((x0 & 0xffffffffull) | (x1 << 32))));
        f |= (uint32_t)x2;
    }
    return stalled;
}

template <class P, int V>
__global__ void __launch_bounds__(P::kCoopThreads) run_coop1d_kernel(
    const InstDesc* __restrict__ descs, const InstCtrl* __restrict__ ctrls, int inst,
    CoopSync* __restrict__ cs, int64_t nsteps, int32_t spin_limit)
{
    using R = typename P::R;
    const InstDesc& d = descs[inst];
    const InstCtrl& c = ctrls[inst];
    const uint32_t G = gridDim.x, b = blockIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int nw = blockDim.x >> 6;
    CoopRec* recs = (CoopRec*)d.partials;                // [parity][G]
    CoopView* views = (CoopView*)(recs + 2 * (size_t)G);
    __shared__ double s_sum[kCoopMaxWaves][10];
    __shared__ double s_sm[kCoopMaxWaves];
    __shared__ uint32_t s_fl[kCoopMaxWaves];
    __shared__ int s_stall;  // this workgroup's wait ran out
    __shared__ uint64_t s_msg[3];
    __shared__ double s_gsrc[3][5];  // a forced source's ghosts at the step's start
    // the solve's control, as every workgroup tracks it
    const double t_end = c.t_end;
    const int64_t max_steps = c.max_steps;
    double t = c.t, dt_cfl = c.dt_cfl, dt_last = c.dt_last;
    int64_t steps = c.steps, nacc = 0;
    int cur = c.cur, status = c.status;
    uint32_t bad = 0;
    bool active = status == 0 && t < t_end && steps < max_steps;
    // Per lane, the sums of the last computed step (acc), of the last
    // accepted one (last) and the source increments of every accepted step
    // (bud); they are folded into the workgroup's records once, when the
    // launch ends, not at every step.
    Acc<R> acc, last;
    acc_init(acc);
    acc_init(last);
    double bud0 = 0.0, bud1 = 0.0;
    int64_t st_c = -1;     // last computed step
    bool cur_ok = false;   // ... and whether this workgroup saw it accepted
    // (a forced source needs the boundary variants: V = 0 or CSPH)
    const bool src = (V == 0 || V == kVariantCsph) && d.bc[0] == kBcSource;
    const double* gsrc = src ? &s_gsrc[0][0] : nullptr;
    if (src) {
        if (threadIdx.x < 3) source_ghost_at(d, t, (int)threadIdx.x, s_gsrc[threadIdx.x]);
        __syncthreads();
    }
    for (int64_t st = 0; st < nsteps && active; st++) {
        const uint32_t gen = (uint32_t)(st + 1);
        double dt = dt_cfl;
        if (t + dt > t_end) dt = t_end - t;
        const typename P::K k = P::make(d, dt);
        acc_init(acc);
        st_c = st;
        cur_ok = false;
        // this wave's run of consecutive segments: the equal share
        // [g S / W, (g + 1) S / W) of the S segments over the launch's W waves
        const int64_t W = (int64_t)G * nw, gw = (int64_t)b * nw + wave;
        const int64_t f0 = gw * d.nstrips / W, f1 = (gw + 1) * d.nstrips / W;
        if (f0 < f1) {
            if constexpr (V == kVariantCsph) {
                if (d.any_bc)
                    march_csph<P, true, true>(d, k, cur, gsrc, 0, lane, acc, f0, f1);
                else
                    march_csph<P, false, true>(d, k, cur, gsrc, 0, lane, acc, f0, f1);
            } else if constexpr (V > 0)
                march1d<P, 0, false, V - 1, true>(d, k, cur, nullptr, 0, lane, acc, f0, f1);
            else if (d.riemann == 1)
                march1d_bc<P, 1, true>(d, k, cur, gsrc, 0, lane, acc, f0, f1);
            else
                march1d_hllc<P, kRecipes, true>(d, k, cur, gsrc, 0, lane, acc, f0, f1);
        }
        acc_finish<P>(acc, k);
        // the barrier needs only the signal speed and the failure flags
        uint32_t fl = acc_flags(acc);
        double sm = (double)acc.smax;
        for (int m = 32; m >= 1; m >>= 1) {
            sm = fmax(sm, lane_xor(sm, lane, m));
            fl |= (uint32_t)__builtin_amdgcn_ds_bpermute(((lane ^ m) & 63) << 2, (int)fl);
        }
        if (lane == 0) {
            s_sm[wave] = sm;
            s_fl[wave] = fl;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double m = 0.0;
            uint32_t f = 0;
            for (int w = 0; w < nw; w++) {
                m = fmax(m, s_sm[w]);
                f |= s_fl[w];
            }
            // publish: three (step << 32 | payload) words in this
            // workgroup's slot -- the low and high halves of its signal speed
            // and its flags
            const uint64_t tag = (uint64_t)gen << 32;
            const uint64_t mb = (uint64_t)__double_as_longlong(m);
            uint64_t* sl = &cs->fslot[st & 1][b][0];
            __hip_atomic_store(sl, tag | (mb & 0xffffffffull), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(sl + 1, tag | (mb >> 32), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(sl + 2, tag | (uint64_t)f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            s_stall = 0;
        }
        __syncthreads();
        // every workgroup takes the step's outcome from all slots itself
        // (lane j of wave 0 reads slot j, ...): the same largest signal speed,
        // union of the flags and next dt in each
        if (wave == 0) {
            // lane j reads slot j and, beyond 64 workgroups, slot j + 64
            double m = 0.0;
            uint32_t f = 0u;
            bool stalled;
            if (G <= 64u)
                stalled = poll_slots<false>(cs->fslot[st & 1], G, gen, lane, spin_limit, m, f);
            else if (G <= 128u)
                stalled = poll_slots<true>(cs->fslot[st & 1], G, gen, lane, spin_limit, m, f);
            else
                stalled = poll_slots4(cs->fslot[st & 1], G, gen, lane, spin_limit, m, f);
            for (int mm = 32; mm >= 1; mm >>= 1) {
                m = fmax(m, lane_xor(m, lane, mm));
                f |= (uint32_t)__builtin_amdgcn_ds_bpermute(((lane ^ mm) & 63) << 2, (int)f);
            }
            if (lane == 0) {
                if (stalled) {
                    __hip_atomic_fetch_or(&cs->stall[0], 1u, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
                    s_stall = 1;
                } else {
                    const uint32_t fb = f & 7u;
                    const double dtc = fb ? dt_cfl : d.cfl * d.h / m;
                    const uint64_t db = (uint64_t)__double_as_longlong(dtc);
                    const uint64_t tag = (uint64_t)gen << 32;
                    s_msg[0] = tag | (db & 0xffffffffull);
                    s_msg[1] = tag | (db >> 32);
                    s_msg[2] = tag | (uint64_t)(fb ? fb << 1 : 1u);
                }
            }
        }
        __syncthreads();
        if (s_stall) break;
        const uint32_t out = (uint32_t)s_msg[2];
        if (out & 1u) {
            // accepted: as accept_step advances the control block
            t = t + dt;
            steps = steps + 1;
            cur ^= 1;
            dt_last = dt;
            dt_cfl = __longlong_as_double(
                (long long)((s_msg[0] & 0xffffffffull) | (s_msg[1] << 32)));
            nacc++;
            active = t < t_end && steps < max_steps;
            bud0 += acc.src[0];
            bud1 += acc.src[1];
            last = acc;
            cur_ok = true;
            // the ghosts of the next step (every wave has marched this one)
            if (src && threadIdx.x < 3) source_ghost_at(d, t, (int)threadIdx.x, s_gsrc[threadIdx.x]);
        } else {
            status = -3;   // NG_EPHYS
            bad = out >> 1;
            active = false;
        }
        __syncthreads();   // s_msg, s_stall and s_gsrc are rewritten in the next step
    }
    // The workgroup's records (lanes, then waves in order): the sums of the
    // last computed step and, when this workgroup did not see that step
    // accepted, of the last accepted one.  The after-kernel folds the records
    // of the last step the most advanced workgroup accepted, found by its
    // parity.
    auto put_rec = [&](const Acc<R>& a, double b0, double b1, int64_t step) {
        double v[10];
        for (int q = 0; q < 5; q++) v[q] = a.tot[q];
        v[5] = b0;
        v[6] = b1;
        v[7] = (double)a.smax;
        v[8] = (double)a.rmin;
        v[9] = (double)a.pmin;
        for (int m = 32; m >= 1; m >>= 1) {
            for (int q = 0; q < 7; q++) v[q] += lane_xor(v[q], lane, m);
            v[7] = fmax(v[7], lane_xor(v[7], lane, m));
            v[8] = fmin(v[8], lane_xor(v[8], lane, m));
            v[9] = fmin(v[9], lane_xor(v[9], lane, m));
        }
        if (lane == 0)
            for (int q = 0; q < 10; q++) s_sum[wave][q] = v[q];
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int w = 1; w < nw; w++) {
                for (int q = 0; q < 7; q++) v[q] += s_sum[w][q];
                v[7] = fmax(v[7], s_sum[w][7]);
                v[8] = fmin(v[8], s_sum[w][8]);
                v[9] = fmin(v[9], s_sum[w][9]);
            }
            CoopRec r;
            for (int q = 0; q < 5; q++) r.tot[q] = v[q];
            r.src[0] = v[5];
            r.src[1] = v[6];
            r.smax = v[7];
            r.rho_min = v[8];
            r.p_min = v[9];
            r.flags = 0u;
            r.step = (uint32_t)step;
            recs[(size_t)(step & 1) * G + b] = r;
        }
        __syncthreads();
    };
    if (st_c >= 0) {
        if (cur_ok) {
            put_rec(acc, bud0, bud1, st_c);
        } else {
            put_rec(acc, bud0 + acc.src[0], bud1 + acc.src[1], st_c);
            if (st_c >= 1) put_rec(last, bud0, bud1, st_c - 1);
        }
    }
    // and its view of the control
    if (threadIdx.x == 0) {
        CoopView w;
        w.t = t;
        w.dt_cfl = dt_cfl;
        w.dt_last = dt_last;
        w.steps = steps;
        w.nacc = nacc;
        w.cur = cur;
        w.status = status;
        w.flags = bad;
        w.pad = 0u;
        views[b] = w;
    }
}

// After a cooperative launch of G workgroups (one workgroup): the most
// advanced view of the control (most steps accepted; a rejection over a
// wait that ran out at the same step) becomes the solve's control, with the
// FP64 totals and extrema of the last accepted step and the source budgets of
// every accepted step folded from the records in workgroup order.  A launch
// whose wait ran out leaves the solve stopped with kStatusStall.
__global__ void __launch_bounds__(256) coop_after_kernel(const InstDesc* __restrict__ descs,
                                                         InstCtrl* __restrict__ ctrls, int inst,
                                                         const CoopSync* __restrict__ cs, int G)
{
    const InstDesc& d = descs[inst];
    InstCtrl& c = ctrls[inst];
    const CoopRec* recs = (const CoopRec*)d.partials;
    const CoopView* views = (const CoopView*)(recs + 2 * (size_t)G);
    __shared__ uint64_t s_key[4];
    __shared__ double sh[4][10];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    // key of a view: steps accepted, then rejection, then the lowest index
    uint64_t key = 0;
    for (int j = t; j < G; j += blockDim.x) {
        const CoopView& a = views[j];
        const uint64_t kj = ((uint64_t)a.nacc << 33) | ((uint64_t)(a.status != 0) << 32) |
                            (uint64_t)(0xffffffffu - (uint32_t)j);
        key = kj > key ? kj : key;
    }
    for (int m = 32; m >= 1; m >>= 1) {
        const int src = ((lane ^ m) & 63) << 2;
        const uint32_t lo = (uint32_t)__builtin_amdgcn_ds_bpermute(src, (int)(uint32_t)key);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_ds_bpermute(src, (int)(uint32_t)(key >> 32));
        const uint64_t o = ((uint64_t)hi << 32) | lo;
        key = o > key ? o : key;
    }
    if (lane == 0) s_key[wave] = key;
    __syncthreads();
    for (int x = 0; x < (int)(blockDim.x >> 6); x++) key = s_key[x] > key ? s_key[x] : key;
    const CoopView w = views[0xffffffffu - (uint32_t)key];
    const int p = (int)((w.nacc - 1) & 1);
    double v[10] = {0, 0, 0, 0, 0, 0, 0, 0, INFINITY, INFINITY};
    if (w.nacc > 0) {
        for (int j = t; j < G; j += blockDim.x) {
            const CoopRec& r = recs[(size_t)p * G + j];
            for (int q = 0; q < 5; q++) v[q] += r.tot[q];
            v[5] += r.src[0];
            v[6] += r.src[1];
            v[7] = fmax(v[7], r.smax);
            v[8] = fmin(v[8], r.rho_min);
            v[9] = fmin(v[9], r.p_min);
        }
        for (int m = 32; m >= 1; m >>= 1) {
            for (int q = 0; q < 7; q++) v[q] += lane_xor(v[q], lane, m);
            v[7] = fmax(v[7], lane_xor(v[7], lane, m));
            v[8] = fmin(v[8], lane_xor(v[8], lane, m));
            v[9] = fmin(v[9], lane_xor(v[9], lane, m));
        }
        if (lane == 0)
            for (int q = 0; q < 10; q++) sh[wave][q] = v[q];
    }
    __syncthreads();
    if (t != 0) return;
    if (w.nacc > 0) {
        for (int x = 1; x < (int)(blockDim.x >> 6); x++) {
            for (int q = 0; q < 7; q++) v[q] += sh[x][q];
            v[7] = fmax(v[7], sh[x][7]);
            v[8] = fmin(v[8], sh[x][8]);
            v[9] = fmin(v[9], sh[x][9]);
        }
        const double n = (double)d.ncell;
        for (int q = 0; q < 5; q++) c.total[q] = v[q] + n * d.uref[q];
        c.budget[0] += v[5];
        c.budget[1] += v[6];
        c.smax = v[7];
        c.rho_min = v[8];
        c.p_min = v[9];
        c.t = w.t;
        c.steps = w.steps;
        c.cur = w.cur;
        c.dt_cfl = w.dt_cfl;
        c.dt_last = w.dt_last;
        c.flags = 0u;
        if (d.bc[0] == kBcSource) source_ghosts(d, c);
    }
    if (w.status != 0) {
        c.status = w.status;
        c.flags = w.flags;
    } else if (cs->stall[0] != 0u && c.status == 0) {
        c.status = kStatusStall;
    }
}

// ======================================================= static scratch

// Device memory of the entry point for callers that cannot allocate
// (ng_step_static): the solve's descriptor and control block, the index list
// of the finalize kernel, the workgroup table and the per-workgroup reduction
// records, in one file-scope array of kStaticScratchBytes that each GPU holds
// until the process ends.  Host code never uses the array's name as an
// address: static_scratch() takes each device's own address of it once.
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

hipError_t static_scratch(void** ptr)
{
    static std::mutex mu;
    static void* addr[kMaxDevices] = {};
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    return hipSuccess;
}

// Fill the static scratch for one solve: descriptor, control block and index
// list from the arguments (no host staging), and the workgroup table
// (workgroup j of the launch is workgroup j of solve 0).
__global__ void static_setup_kernel(InstDesc d, InstCtrl c, InstDesc* __restrict__ descs,
                                    InstCtrl* __restrict__ ctrls, int32_t* __restrict__ insts,
                                    BlockRef* __restrict__ blocks, int64_t nblocks)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        descs[0] = d;
        ctrls[0] = c;
        insts[0] = 0;
    }
    for (; i < nblocks; i += (int64_t)gridDim.x * blockDim.x) blocks[i] = BlockRef{0, (int32_t)i};
}

hipError_t launch_static_setup(const InstDesc& d, const InstCtrl& c, InstDesc* descs,
                               InstCtrl* ctrls, int32_t* insts, BlockRef* blocks,
                               int64_t nblocks, hipStream_t s)
{
    const int64_t g = nblocks < 256 * 64 ? (nblocks + 255) / 256 : 64;
    hipLaunchKernelGGL(static_setup_kernel, dim3((unsigned)(g > 0 ? g : 1)), dim3(256), 0, s, d,
                       c, descs, ctrls, insts, blocks, nblocks);
    return hipGetLastError();
}

// ================================================================ launchers

static inline bool grid_ok(int64_t nblocks) { return nblocks > 0 && nblocks < (1LL << 31); }

// Launch on s; with events, through the AMD extension that records the
// kernel's own start and end in them (no separate event packets on the
// stream, so timing adds no gaps between launches).  Untimed launches use the
// plain form, which stream capture records as a kernel node.
template <class... A>
static void launch(void (*kernel)(A...), dim3 g, dim3 b, hipStream_t s, hipEvent_t e0,
                   hipEvent_t e1, A... a)
{
    if (e0 || e1)
        hipExtLaunchKernelGGL(kernel, g, b, 0, s, e0, e1, 0, a...);
    else
        hipLaunchKernelGGL(kernel, g, b, 0, s, a...);
}

// Step kernel of a policy for variant v (the FP64 arithmetic has no closure
// recipes: its periodic-HLLC variant is 1 whatever the recipe).
template <template <int> class Pol, int NC>
static void launch_variant(int v, dim3 g, dim3 b, hipStream_t s, hipEvent_t e0, hipEvent_t e1,
                           const InstDesc* descs, InstCtrl* ctrls, const BlockRef* blocks,
                           int remap, int fused)
{
    using P = Pol<NC>;
    if constexpr (NC == 5) {
        if (v == 0) launch(step2d_kernel<P, 0>, g, b, s, e0, e1, descs, ctrls, blocks, remap, fused);
        else if (v == 1 || !P::kRecipes)
            launch(step2d_kernel<P, 1>, g, b, s, e0, e1, descs, ctrls, blocks, remap, fused);
        else if constexpr (P::kRecipes) {
            if (v == 2) launch(step2d_kernel<P, 2>, g, b, s, e0, e1, descs, ctrls, blocks, remap, fused);
            else launch(step2d_kernel<P, 3>, g, b, s, e0, e1, descs, ctrls, blocks, remap, fused);
        }
    } else {
        if (v == 0) launch(step1d_kernel<P, 0>, g, b, s, e0, e1, descs, ctrls, blocks, remap, fused);
        else if constexpr (std::is_same<typename P::K, K64>::value) {
            if (v == kVariantCsph)
                launch(step1d_kernel<P, kVariantCsph>, g, b, s, e0, e1, descs, ctrls, blocks, remap,
                       fused);
            else
                launch(step1d_kernel<P, 1>, g, b, s, e0, e1, descs, ctrls, blocks, remap, fused);
        } else if (v == 1 || !P::kRecipes)
            launch(step1d_kernel<P, 1>, g, b, s, e0, e1, descs, ctrls, blocks, remap, fused);
        else if constexpr (P::kRecipes) {
            if (v == 2) launch(step1d_kernel<P, 2>, g, b, s, e0, e1, descs, ctrls, blocks, remap, fused);
            else launch(step1d_kernel<P, 3>, g, b, s, e0, e1, descs, ctrls, blocks, remap, fused);
        }
    }
}

hipError_t launch_step(int dim, int prec, int variant, const InstDesc* descs, InstCtrl* ctrls,
                       const BlockRef* blocks, int64_t nblocks, int waves, int remap, int fused,
                       hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    static_assert(kRecipes == 2, "launch_variant instantiates variants 0..3");
    if (!grid_ok(nblocks) || waves < 1 || waves > 4) return hipErrorInvalidValue;
    if (variant < 0 || (variant > kRecipes + 1 &&
                        !(variant == kVariantCsph && dim == 1 && prec == 0)))
        return hipErrorInvalidValue;
    dim3 g((unsigned)nblocks), b((unsigned)(64 * waves));
    if (dim == 2) {
        if (prec == 0)
            launch_variant<Plain64, 5>(variant, g, b, s, e0, e1, descs, ctrls, blocks, remap, fused);
        else if (prec == 1)
            launch_variant<Dev32, 5>(variant, g, b, s, e0, e1, descs, ctrls, blocks, remap, fused);
        else
            launch_variant<Mix32, 5>(variant, g, b, s, e0, e1, descs, ctrls, blocks, remap, fused);
    } else {
        if (prec == 0)
            launch_variant<Plain64, 4>(variant, g, b, s, e0, e1, descs, ctrls, blocks, remap, fused);
        else if (prec == 1)
            launch_variant<Dev32, 4>(variant, g, b, s, e0, e1, descs, ctrls, blocks, remap, fused);
        else
            launch_variant<Mix32, 4>(variant, g, b, s, e0, e1, descs, ctrls, blocks, remap, fused);
    }
    return hipGetLastError();
}

hipError_t launch_prime(int dim, int prec, const InstDesc* descs, InstCtrl* ctrls,
                        const BlockRef* blocks, int inst, int64_t nblocks, int waves,
                        hipStream_t s)
{
    if (!grid_ok(nblocks) || waves < 1 || waves > 4) return hipErrorInvalidValue;
    dim3 g((unsigned)nblocks), b((unsigned)(64 * waves));
    if (dim == 2) {
        if (prec == 0)
            hipLaunchKernelGGL((prime_kernel<Plain64<5>, 5>), g, b, 0, s, descs, ctrls, blocks, inst);
        else if (prec == 1)
            hipLaunchKernelGGL((prime_kernel<Dev32<5>, 5>), g, b, 0, s, descs, ctrls, blocks, inst);
        else
            hipLaunchKernelGGL((prime_kernel<Mix32<5>, 5>), g, b, 0, s, descs, ctrls, blocks, inst);
    } else {
        if (prec == 0)
            hipLaunchKernelGGL((prime_kernel<Plain64<4>, 4>), g, b, 0, s, descs, ctrls, blocks, inst);
        else if (prec == 1)
            hipLaunchKernelGGL((prime_kernel<Dev32<4>, 4>), g, b, 0, s, descs, ctrls, blocks, inst);
        else
            hipLaunchKernelGGL((prime_kernel<Mix32<4>, 4>), g, b, 0, s, descs, ctrls, blocks, inst);
    }
    return hipGetLastError();
}

hipError_t launch_finalize(const InstDesc* descs, InstCtrl* ctrls, const int32_t* insts, int n,
                           int mode, hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    if (n <= 0) return hipSuccess;
    // four waves per solve: enough to fold a few thousand records with one
    // load in flight per lane, and a quarter of the dispatch work of 1024
    // threads when a batch finalizes hundreds of solves (512 solves: 108 ->
    // 99 us per step; 4096^2 alone: 10.8 -> 8.0 us)
    launch(finalize_kernel, dim3((unsigned)n), dim3(256), s, e0, e1, descs, ctrls, insts, mode);
    return hipGetLastError();
}

hipError_t launch_small(int dim, int prec, const InstDesc* descs, InstCtrl* ctrls,
                        const int32_t* insts, int n, int waves, int64_t nsteps, hipStream_t s)
{
    if (n <= 0 || nsteps <= 0) return hipSuccess;
    if (waves < 1 || waves > kMaxWaves) return hipErrorInvalidValue;
    dim3 g((unsigned)n), b((unsigned)(64 * waves));
    if (dim == 2) {
        if (prec == 0)
            hipLaunchKernelGGL((run_small_kernel<Plain64<5>, 5>), g, b, 0, s, descs, ctrls, insts, nsteps);
        else if (prec == 1)
            hipLaunchKernelGGL((run_small_kernel<Dev32<5>, 5>), g, b, 0, s, descs, ctrls, insts, nsteps);
        else
            hipLaunchKernelGGL((run_small_kernel<Mix32<5>, 5>), g, b, 0, s, descs, ctrls, insts, nsteps);
    } else {
        if (prec == 0)
            hipLaunchKernelGGL((run_small_kernel<Plain64<4>, 4>), g, b, 0, s, descs, ctrls, insts, nsteps);
        else if (prec == 1)
            hipLaunchKernelGGL((run_small_kernel<Dev32<4>, 4>), g, b, 0, s, descs, ctrls, insts, nsteps);
        else
            hipLaunchKernelGGL((run_small_kernel<Mix32<4>, 4>), g, b, 0, s, descs, ctrls, insts, nsteps);
    }
    return hipGetLastError();
}

// The cooperative 1D kernel of a precision and variant (as launch_step).
template <template <int> class Pol>
static const void* coop_kernel_of(int v)
{
    using P = Pol<4>;
    if (v == 0) return (const void*)run_coop1d_kernel<P, 0>;
    if constexpr (std::is_same<typename P::K, K64>::value) {
        if (v == kVariantCsph) return (const void*)run_coop1d_kernel<P, kVariantCsph>;
    }
    if (v == 1 || !P::kRecipes) return (const void*)run_coop1d_kernel<P, 1>;
    if constexpr (P::kRecipes) {
        if (v == 2) return (const void*)run_coop1d_kernel<P, 2>;
        return (const void*)run_coop1d_kernel<P, 3>;
    }
    return nullptr;
}

static const void* coop_kernel(int prec, int variant)
{
    if (variant < 0 || (variant > kRecipes + 1 && !(variant == kVariantCsph && prec == 0)))
        return nullptr;
    if (prec == 0) return coop_kernel_of<Plain64>(variant);
    if (prec == 1) return coop_kernel_of<Dev32>(variant);
    if (prec == 2) return coop_kernel_of<Mix32>(variant);
    return nullptr;
}

static int coop_max_threads(int prec)
{
    return prec == 0 ? Plain64<4>::kCoopThreads
                     : (prec == 1 ? Dev32<4>::kCoopThreads : Mix32<4>::kCoopThreads);
}

hipError_t coop_capacity(int prec, int variant, int waves, int* blocks_per_cu, int* max_waves)
{
    const void* k = coop_kernel(prec, variant);
    if (!k) return hipErrorInvalidValue;
    *max_waves = coop_max_threads(prec) / kWave;
    if (waves < 1 || waves > *max_waves) return hipErrorInvalidValue;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k, waves * kWave, 0);
}

hipError_t launch_coop(int prec, int variant, const InstDesc* descs, InstCtrl* ctrls, int inst,
                       CoopSync* cs, int grid, int waves, int64_t nsteps, int32_t spin_limit,
                       hipStream_t s)
{
    const void* k = coop_kernel(prec, variant);
    const int maxw = coop_max_threads(prec) / kWave;
    if (!k || grid < 1 || waves < 1 || waves > maxw || nsteps < 1 || nsteps > kCoopMaxSteps ||
        spin_limit < 0)
        return hipErrorInvalidValue;
    hipError_t e = hipMemsetAsync(cs, 0, sizeof(CoopSync), s);
    if (e != hipSuccess) return e;
    void* args[] = {(void*)&descs, (void*)&ctrls, (void*)&inst, (void*)&cs, (void*)&nsteps,
                    (void*)&spin_limit};
    e = hipLaunchCooperativeKernel(k, dim3((unsigned)grid), dim3((unsigned)(waves * kWave)), args,
                                   0, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(coop_after_kernel, dim3(1), dim3(256), 0, s, descs, ctrls, inst,
                       (const CoopSync*)cs, grid);
    return hipGetLastError();
}

hipError_t launch_set_limits(InstCtrl* ctrls, const int32_t* insts, int n, double t_end,
                             int64_t max_steps_from_now, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(set_limits_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       ctrls, insts, n, t_end, max_steps_from_now);
    return hipGetLastError();
}

}  // namespace ng
