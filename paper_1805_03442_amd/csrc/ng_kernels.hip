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
//   1D: a work item is a group of consecutive 60-cell segments.
// Each cell's arithmetic does not depend on where it sits in a strip or chunk,
// so results are independent of the launch shape.
//
// The step kernel writes U^{n+1} into the other state buffer and, per
// workgroup, the max signal speed of U^{n+1}, the FP64 sums of U^{n+1}, the
// FP64 sums of the source increments, minima of rho and p and failure flags.
// The finalize kernel (one workgroup per solve) folds those records in a fixed
// order, accepts or rejects the step, advances t and computes the next dt.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "ng_cell.hpp"
#include "ng_internal.hpp"
#include "ng_launch.hpp"

namespace ng {

// ------------------------------------------------------------ cross-lane

__device__ __forceinline__ float lane_get(float v, int addr)
{
    return __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(v)));
}
__device__ __forceinline__ double lane_get(double v, int addr)
{
    int lo = __double2loint(v), hi = __double2hiint(v);
    lo = __builtin_amdgcn_ds_bpermute(addr, lo);
    hi = __builtin_amdgcn_ds_bpermute(addr, hi);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double lane_xor(double v, int lane, int m)
{
    return lane_get(v, ((lane ^ m) & 63) << 2);
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
    static __device__ void predict(const K& k, const R* W, const R* sx, const R* sy, R* Wh)
    {
        predict64<NC>(k, W, sx, sy, Wh);
    }
    static __device__ void flux(const K& k, const R* L, const R* Rr, R* F) { flux64<NC>(k, L, Rr, F); }
    static __device__ void update(const K& k, const R* Un, const R* dF, const R* dG, const R* Wh,
                                  R* Unew, R& sE, R& sV)
    {
        update64<NC>(k, Un, dF, dG, Wh, Unew, sE, sV);
    }
    static __device__ R half() { return 0.5; }
    static __device__ double full_rho(const K&, R r) { return r; }
    static __device__ double full_p(const K&, R p) { return p; }
};

template <int NC>
struct Dev32 {
    using R = float;
    using K = K32;
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
        k.irho0 = (float)(1.0 / d.rho0);
        k.iRT0 = (float)(1.0 / (d.R * d.T0));
        k.itau0 = (float)(1.0 / d.tau0);
        k.Q0 = (float)d.Q0;
        k.I0 = (float)d.I0;
        k.tr = (float)d.tau_rho;
        k.tT = (float)d.tau_T;
        k.Qr = (float)d.Q_rho;
        k.QT = (float)d.Q_T;
        k.Ir = (float)d.I_rho;
        k.IT = (float)d.I_T;
        k.fx = (float)d.fx;
        k.fy = (float)d.fy;
        k.stiff_z = (float)d.stiff_z;
        k.dt = (float)dt;
        k.dtdx = (float)(dt / d.h);
        k.hdtdx = 0.5f * k.dtdx;
        k.hdt = 0.5f * k.dt;
        k.dt64 = (double)k.dt;
        k.hdt64 = (double)k.hdt;
        k.riemann = d.riemann;
        return k;
    }
    static __device__ void prim(const K& k, const R* U, R* W) { prim32<NC>(k, U, W); }
    static __device__ R speed(const K& k, const R* W) { return speed32<NC>(k, W); }
    static __device__ void predict(const K& k, const R* W, const R* sx, const R* sy, R* Wh)
    {
        predict32<NC>(k, W, sx, sy, Wh);
    }
    static __device__ void flux(const K& k, const R* L, const R* Rr, R* F) { flux32<NC>(k, L, Rr, F); }
    static __device__ void update(const K& k, const R* Un, const R* dF, const R* dG, const R* Wh,
                                  R* Unew, R& sE, R& sV)
    {
        update32<NC>(k, Un, dF, dG, Wh, Unew, sE, sV);
    }
    static __device__ R half() { return 0.5f; }
    static __device__ double full_rho(const K& k, R r) { return (double)(k.rho_r + r); }
    static __device__ double full_p(const K& k, R p) { return (double)(k.p_r + p); }
};

// ------------------------------------------------------ reduction records

struct Acc {
    double tot[5];
    double src[2];
    double smax, rmin, pmin;
    uint32_t flags;
};

__device__ __forceinline__ void acc_init(Acc& a)
{
    for (int c = 0; c < 5; c++) a.tot[c] = 0.0;
    a.src[0] = a.src[1] = 0.0;
    a.smax = 0.0;
    a.rmin = INFINITY;
    a.pmin = INFINITY;
    a.flags = 0u;
}

// Record one updated cell: NC conserved values (as stored), its primitives
// and signal speed, and its source increments.
template <class P, int NC>
__device__ __forceinline__ void acc_cell(Acc& a, const typename P::K& k,
                                         const typename P::R* U, const typename P::R* W,
                                         typename P::R s, typename P::R sE, typename P::R sV)
{
    // component slots (rho, m_x, m_y, E, E_nu)
    if (NC == 5) {
        for (int c = 0; c < 5; c++) a.tot[c] += (double)U[c];
    } else {
        a.tot[0] += (double)U[0];
        a.tot[1] += (double)U[1];
        a.tot[3] += (double)U[2];
        a.tot[4] += (double)U[3];
    }
    a.src[0] += (double)sE;
    a.src[1] += (double)sV;
    double rho = P::full_rho(k, W[0]);
    double p = P::full_p(k, W[NC == 5 ? 3 : 2]);
    double sd = (double)s;
    a.smax = sd > a.smax ? sd : a.smax;
    a.rmin = rho < a.rmin ? rho : a.rmin;
    a.pmin = p < a.pmin ? p : a.pmin;
    bool fin = true;
    for (int c = 0; c < NC; c++) fin = fin && isfinite(U[c]);
    fin = fin && isfinite(sd);
    if (!fin) a.flags |= 1u;
    if (!(rho > 0.0)) a.flags |= 2u;
    if (!(p > 0.0)) a.flags |= 4u;
}

// Fold the lanes of each wave (lane 0 keeps a fixed-order result), then the
// waves of the workgroup in wave order, and store the workgroup's record.
__device__ void block_reduce_store(Acc& a, Partial* out, int wave, int lane, int nwaves)
{
    __shared__ double sh[kMaxWaves][11];
    __shared__ uint32_t shf[kMaxWaves];
    for (int m = 32; m >= 1; m >>= 1) {
        for (int c = 0; c < 5; c++) a.tot[c] += lane_xor(a.tot[c], lane, m);
        a.src[0] += lane_xor(a.src[0], lane, m);
        a.src[1] += lane_xor(a.src[1], lane, m);
        double o = lane_xor(a.smax, lane, m);
        a.smax = o > a.smax ? o : a.smax;
        o = lane_xor(a.rmin, lane, m);
        a.rmin = o < a.rmin ? o : a.rmin;
        o = lane_xor(a.pmin, lane, m);
        a.pmin = o < a.pmin ? o : a.pmin;
        a.flags |= (uint32_t)__builtin_amdgcn_ds_bpermute(((lane ^ m) & 63) << 2, (int)a.flags);
    }
    if (lane == 0) {
        for (int c = 0; c < 5; c++) sh[wave][c] = a.tot[c];
        sh[wave][5] = a.src[0];
        sh[wave][6] = a.src[1];
        sh[wave][7] = a.smax;
        sh[wave][8] = a.rmin;
        sh[wave][9] = a.pmin;
        shf[wave] = a.flags;
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
            r.smax = sh[w][7] > r.smax ? sh[w][7] : r.smax;
            r.rho_min = sh[w][8] < r.rho_min ? sh[w][8] : r.rho_min;
            r.p_min = sh[w][9] < r.p_min ? sh[w][9] : r.p_min;
            r.flags |= shf[w];
        }
        *out = r;
    }
}

// Control word of a solve as seen by the kernels of one step.
struct StepCtl {
    double dt;
    int cur;
    bool active;
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
    return s;
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

// ================================================================ 2D step

template <class P>
__global__ void __launch_bounds__(256) step2d_kernel(const InstDesc* __restrict__ descs,
                                                     InstCtrl* __restrict__ ctrls,
                                                     const BlockRef* __restrict__ blocks,
                                                     int remap)
{
    using R = typename P::R;
    constexpr int NC = 5;
    const int64_t G = gridDim.x;
    const int64_t bid = remap ? xcd_remap(blockIdx.x, G) : (int64_t)blockIdx.x;
    const BlockRef br = blocks[bid];
    const InstDesc& d = descs[br.inst];
    const StepCtl sc = read_ctl(ctrls[br.inst]);
    if (!sc.active) return;
    const typename P::K k = P::make(d, sc.dt);
    const R half = P::half();

    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int al = ((lane + 63) & 63) << 2, ar = ((lane + 1) & 63) << 2;
    const int nwaves = d.waves_per_block;
    Acc acc;
    acc_init(acc);

    const int64_t item = (int64_t)br.local * nwaves + wave;
    if (item < d.nitems) {
        const int64_t nx = d.nx, ny = d.ny, ncell = d.ncell;
        const int64_t strip = item % d.nstrips, chunk = item / d.nstrips;
        const int64_t x0 = strip * kInterior;
        int64_t x = x0 - kHalo + lane;
        x = ((x % nx) + nx) % nx;
        const bool inner = lane >= kHalo && lane < kWave - kHalo && x0 + (lane - kHalo) < nx;
        const int64_t r0 = chunk * d.rows_per_item;
        const int64_t r1 = r0 + d.rows_per_item < ny ? r0 + d.rows_per_item : ny;
        const R* __restrict__ src = (const R*)d.buf[sc.cur];
        R* __restrict__ dst = (R*)d.buf[sc.cur ^ 1];
        auto rowi = [&](int64_t r) -> int64_t {
            int64_t rr = ((r % ny) + ny) % ny;
            return rr * nx + x;
        };

        R Wc[NC], Wd[NC], We[NC], Ut[NC], Un[NC];
        R h0[NC], sx0[NC], Nprev[NC], Gprev[NC];
        R sx[NC], sy[NC], h1[NC], Wl[NC], Wr[NC];

        // prologue: rows r0-2 .. r0+1, the half-step state of rows r0-1 and r0
        {
            R Wa[NC], Wb[NC];
            load_cell<R, NC>(src, ncell, rowi(r0 - 2), Ut);
            P::prim(k, Ut, Wa);
            load_cell<R, NC>(src, ncell, rowi(r0 - 1), Ut);
            P::prim(k, Ut, Wb);
            load_cell<R, NC>(src, ncell, rowi(r0), Ut);
            P::prim(k, Ut, Wc);
            load_cell<R, NC>(src, ncell, rowi(r0 + 1), Ut);
            P::prim(k, Ut, Wd);
            // row r0-1
            for (int c = 0; c < NC; c++) {
                Wl[c] = lane_get(Wb[c], al);
                Wr[c] = lane_get(Wb[c], ar);
                sx[c] = minmod(Wb[c] - Wl[c], Wr[c] - Wb[c]);
                sy[c] = minmod(Wb[c] - Wa[c], Wc[c] - Wb[c]);
            }
            P::predict(k, Wb, sx, sy, h1);
            for (int c = 0; c < NC; c++) Nprev[c] = h1[c] + half * sy[c];
            // row r0
            for (int c = 0; c < NC; c++) {
                Wl[c] = lane_get(Wc[c], al);
                Wr[c] = lane_get(Wc[c], ar);
                sx0[c] = minmod(Wc[c] - Wl[c], Wr[c] - Wc[c]);
                sy[c] = minmod(Wc[c] - Wb[c], Wd[c] - Wc[c]);
            }
            P::predict(k, Wc, sx0, sy, h0);
            R S[NC], Nr[NC], Sr[NC], Fy[NC];
            for (int c = 0; c < NC; c++) S[c] = h0[c] - half * sy[c];
            // y-face r0-1/2: normal velocity is v -> swap (u, v)
            Nr[0] = Nprev[0]; Nr[1] = Nprev[2]; Nr[2] = Nprev[1]; Nr[3] = Nprev[3]; Nr[4] = Nprev[4];
            Sr[0] = S[0]; Sr[1] = S[2]; Sr[2] = S[1]; Sr[3] = S[3]; Sr[4] = S[4];
            P::flux(k, Nr, Sr, Fy);
            Gprev[0] = Fy[0]; Gprev[1] = Fy[2]; Gprev[2] = Fy[1]; Gprev[3] = Fy[3]; Gprev[4] = Fy[4];
            for (int c = 0; c < NC; c++) Nprev[c] = h0[c] + half * sy[c];
        }
        load_cell<R, NC>(src, ncell, rowi(r0 + 2), Ut);   // prefetched row

        for (int64_t i = r0; i < r1; i++) {
            // row i+2 arrives; issue row i+3
            for (int c = 0; c < NC; c++) Un[c] = Ut[c];
            P::prim(k, Un, We);
            if (i + 1 < r1) load_cell<R, NC>(src, ncell, rowi(i + 3), Ut);

            // predictor of row i+1
            for (int c = 0; c < NC; c++) {
                Wl[c] = lane_get(Wd[c], al);
                Wr[c] = lane_get(Wd[c], ar);
                sx[c] = minmod(Wd[c] - Wl[c], Wr[c] - Wd[c]);
                sy[c] = minmod(Wd[c] - Wc[c], We[c] - Wd[c]);
            }
            P::predict(k, Wd, sx, sy, h1);

            // y-face i+1/2
            R Gn[NC];
            {
                R Nr[NC], Sr[NC], Fy[NC];
                Nr[0] = Nprev[0]; Nr[1] = Nprev[2]; Nr[2] = Nprev[1]; Nr[3] = Nprev[3]; Nr[4] = Nprev[4];
                Sr[0] = h1[0] - half * sy[0];
                Sr[1] = h1[2] - half * sy[2];
                Sr[2] = h1[1] - half * sy[1];
                Sr[3] = h1[3] - half * sy[3];
                Sr[4] = h1[4] - half * sy[4];
                P::flux(k, Nr, Sr, Fy);
                Gn[0] = Fy[0]; Gn[1] = Fy[2]; Gn[2] = Fy[1]; Gn[3] = Fy[3]; Gn[4] = Fy[4];
            }

            // x-faces of row i: lane j computes face j+1/2 from its east state
            // and lane j+1's west state; face j-1/2 comes from lane j-1
            R dF[NC], dG[NC];
            {
                R E[NC], Wf[NC], Fx[NC];
                for (int c = 0; c < NC; c++) {
                    E[c] = h0[c] + half * sx0[c];
                    Wf[c] = h0[c] - half * sx0[c];
                }
                for (int c = 0; c < NC; c++) Wr[c] = lane_get(Wf[c], ar);
                P::flux(k, E, Wr, Fx);
                for (int c = 0; c < NC; c++) {
                    R Fl = lane_get(Fx[c], al);
                    dF[c] = Fx[c] - Fl;
                    dG[c] = Gn[c] - Gprev[c];
                }
            }

            // update of row i
            R Uo[NC], Wn[NC], sE, sV;
            const int64_t idx = rowi(i);
            load_cell_cached<R, NC>(src, ncell, idx, Un);
            P::update(k, Un, dF, dG, h0, Uo, sE, sV);
            P::prim(k, Uo, Wn);
            R s = P::speed(k, Wn);
            if (inner) {
                for (int c = 0; c < NC; c++) __builtin_nontemporal_store(Uo[c], dst + c * ncell + idx);
                acc_cell<P, NC>(acc, k, Uo, Wn, s, sE, sV);
            }

            // rotate the rolling window
            for (int c = 0; c < NC; c++) {
                Gprev[c] = Gn[c];
                Nprev[c] = h1[c] + half * sy[c];
                h0[c] = h1[c];
                sx0[c] = sx[c];
                Wc[c] = Wd[c];
                Wd[c] = We[c];
            }
        }
    }
    Partial* parts = (Partial*)d.partials;
    block_reduce_store(acc, parts + br.local, wave, lane, nwaves);
}

// ================================================================ 1D step

template <class P>
__global__ void __launch_bounds__(256) step1d_kernel(const InstDesc* __restrict__ descs,
                                                     InstCtrl* __restrict__ ctrls,
                                                     const BlockRef* __restrict__ blocks,
                                                     int remap)
{
    using R = typename P::R;
    constexpr int NC = 4;
    const int64_t G = gridDim.x;
    const int64_t bid = remap ? xcd_remap(blockIdx.x, G) : (int64_t)blockIdx.x;
    const BlockRef br = blocks[bid];
    const InstDesc& d = descs[br.inst];
    const StepCtl sc = read_ctl(ctrls[br.inst]);
    if (!sc.active) return;
    const typename P::K k = P::make(d, sc.dt);
    const R half = P::half();

    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int al = ((lane + 63) & 63) << 2, ar = ((lane + 1) & 63) << 2;
    const int nwaves = d.waves_per_block;
    Acc acc;
    acc_init(acc);

    const int64_t item = (int64_t)br.local * nwaves + wave;
    if (item < d.nitems) {
        const int64_t n = d.nx;
        const R* __restrict__ src = (const R*)d.buf[sc.cur];
        R* __restrict__ dst = (R*)d.buf[sc.cur ^ 1];
        const int64_t s0 = item * d.rows_per_item;
        const int64_t s1 = s0 + d.rows_per_item < d.nstrips ? s0 + d.rows_per_item : d.nstrips;
        auto cell = [&](int64_t sg) -> int64_t {
            int64_t xx = sg * kInterior - kHalo + lane;
            return ((xx % n) + n) % n;
        };
        R Ut[NC];
        load_cell<R, NC>(src, n, cell(s0), Ut);
        for (int64_t sg = s0; sg < s1; sg++) {
            R Un[NC], W[NC], Wl[NC], Wr[NC], sx[NC], h[NC];
            for (int c = 0; c < NC; c++) Un[c] = Ut[c];
            const int64_t idx = cell(sg);
            if (sg + 1 < s1) load_cell<R, NC>(src, n, cell(sg + 1), Ut);
            P::prim(k, Un, W);
            for (int c = 0; c < NC; c++) {
                Wl[c] = lane_get(W[c], al);
                Wr[c] = lane_get(W[c], ar);
                sx[c] = minmod(W[c] - Wl[c], Wr[c] - W[c]);
            }
            P::predict(k, W, sx, sx, h);
            R E[NC], Wf[NC], Fx[NC], dF[NC];
            for (int c = 0; c < NC; c++) {
                E[c] = h[c] + half * sx[c];
                Wf[c] = h[c] - half * sx[c];
            }
            for (int c = 0; c < NC; c++) Wr[c] = lane_get(Wf[c], ar);
            P::flux(k, E, Wr, Fx);
            for (int c = 0; c < NC; c++) dF[c] = Fx[c] - lane_get(Fx[c], al);
            R Uo[NC], Wn[NC], sE, sV;
            P::update(k, Un, dF, dF, h, Uo, sE, sV);
            P::prim(k, Uo, Wn);
            R s = P::speed(k, Wn);
            const bool inner = lane >= kHalo && lane < kWave - kHalo &&
                               sg * kInterior + (lane - kHalo) < n;
            if (inner) {
                for (int c = 0; c < NC; c++) __builtin_nontemporal_store(Uo[c], dst + c * n + idx);
                acc_cell<P, NC>(acc, k, Uo, Wn, s, sE, sV);
            }
        }
    }
    Partial* parts = (Partial*)d.partials;
    block_reduce_store(acc, parts + br.local, wave, lane, nwaves);
}

// ============================================================ priming pass

// Signal speed, sums and checks of the current state (no step): the records
// from which the finalize kernel derives the first dt and the totals.
template <class P, int NC>
__global__ void __launch_bounds__(256) prime_kernel(const InstDesc* __restrict__ descs,
                                                    InstCtrl* __restrict__ ctrls,
                                                    const BlockRef* __restrict__ blocks)
{
    using R = typename P::R;
    const BlockRef br = blocks[blockIdx.x];
    const InstDesc& d = descs[br.inst];
    const InstCtrl& cc = ctrls[br.inst];
    if (cc.status != 0) return;
    const typename P::K k = P::make(d, 0.0);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nwaves = d.waves_per_block;
    Acc acc;
    acc_init(acc);
    const int64_t item = (int64_t)br.local * nwaves + wave;
    if (item < d.nitems) {
        const R* __restrict__ src = (const R*)d.buf[cc.cur];
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
        for (int64_t sg = seg0; sg < seg1; sg++) {
            const int64_t xbase = NC == 5 ? xs : sg * kInterior;
            const int64_t xo = xbase + (lane - kHalo);
            const bool inner = lane >= kHalo && lane < kWave - kHalo && xo < nx;
            if (!inner) continue;
            for (int64_t r = rows0; r < rows1; r++) {
                R U[NC], W[NC];
                load_cell_cached<R, NC>(src, ncell, r * nx + xo, U);
                P::prim(k, U, W);
                R s = P::speed(k, W);
                acc_cell<P, NC>(acc, k, U, W, s, (R)0, (R)0);
            }
        }
    }
    Partial* parts = (Partial*)d.partials;
    block_reduce_store(acc, parts + br.local, wave, lane, nwaves);
}

// ================================================================ finalize

// One workgroup per solve: fold the step's records in a fixed order, accept
// (swap buffers, advance t, next dt from eq. (16)) or reject (sticky NG_EPHYS,
// the state before the step is kept).  mode 0: after a step; 1: priming.
__global__ void __launch_bounds__(256) finalize_kernel(const InstDesc* __restrict__ descs,
                                                       InstCtrl* __restrict__ ctrls,
                                                       const int32_t* __restrict__ insts,
                                                       int mode)
{
    const int inst = insts[blockIdx.x];
    const InstDesc& d = descs[inst];
    InstCtrl& c = ctrls[inst];
    const StepCtl sc = read_ctl(c);
    if (mode == 0 && !sc.active) return;
    if (mode == 1 && c.status != 0) return;
    const Partial* parts = (const Partial*)d.partials;
    const int64_t nb = d.nblocks;
    __shared__ double sh[256][10];
    __shared__ uint32_t shf[256];
    double tot[5] = {0, 0, 0, 0, 0}, src0 = 0.0, src1 = 0.0, smax = 0.0, rmin = INFINITY,
           pmin = INFINITY;
    uint32_t flags = 0;
    for (int64_t b = threadIdx.x; b < nb; b += blockDim.x) {
        const Partial& p = parts[b];
        for (int q = 0; q < 5; q++) tot[q] += p.tot[q];
        src0 += p.src[0];
        src1 += p.src[1];
        smax = p.smax > smax ? p.smax : smax;
        rmin = p.rho_min < rmin ? p.rho_min : rmin;
        pmin = p.p_min < pmin ? p.p_min : pmin;
        flags |= p.flags;
    }
    const int t = threadIdx.x;
    for (int q = 0; q < 5; q++) sh[t][q] = tot[q];
    sh[t][5] = src0;
    sh[t][6] = src1;
    sh[t][7] = smax;
    sh[t][8] = rmin;
    sh[t][9] = pmin;
    shf[t] = flags;
    __syncthreads();
    for (int w = blockDim.x / 2; w >= 1; w >>= 1) {
        if (t < w) {
            for (int q = 0; q < 7; q++) sh[t][q] += sh[t + w][q];
            sh[t][7] = sh[t + w][7] > sh[t][7] ? sh[t + w][7] : sh[t][7];
            sh[t][8] = sh[t + w][8] < sh[t][8] ? sh[t + w][8] : sh[t][8];
            sh[t][9] = sh[t + w][9] < sh[t][9] ? sh[t + w][9] : sh[t][9];
            shf[t] |= shf[t + w];
        }
        __syncthreads();
    }
    if (t != 0) return;
    const double n = (double)d.ncell;
    const uint32_t bad = shf[0] & 7u;
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
        c.budget[0] += sh[0][5];
        c.budget[1] += sh[0][6];
    }
    for (int q = 0; q < 5; q++) c.total[q] = sh[0][q] + n * d.uref[q];
    c.smax = sh[0][7];
    c.rho_min = sh[0][8];
    c.p_min = sh[0][9];
    c.dt_cfl = d.cfl * d.h / sh[0][7];
    c.flags = 0u;
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

// ================================================================ launchers

static inline bool grid_ok(int64_t nblocks) { return nblocks > 0 && nblocks < (1LL << 31); }

hipError_t launch_step(int dim, int prec, const InstDesc* descs, InstCtrl* ctrls,
                       const BlockRef* blocks, int64_t nblocks, int waves, int remap,
                       hipStream_t s)
{
    if (!grid_ok(nblocks) || waves < 1 || waves > 4) return hipErrorInvalidValue;
    dim3 g((unsigned)nblocks), b((unsigned)(64 * waves));
    if (dim == 2) {
        if (prec == 0)
            hipLaunchKernelGGL(step2d_kernel<Plain64<5>>, g, b, 0, s, descs, ctrls, blocks, remap);
        else
            hipLaunchKernelGGL(step2d_kernel<Dev32<5>>, g, b, 0, s, descs, ctrls, blocks, remap);
    } else {
        if (prec == 0)
            hipLaunchKernelGGL(step1d_kernel<Plain64<4>>, g, b, 0, s, descs, ctrls, blocks, remap);
        else
            hipLaunchKernelGGL(step1d_kernel<Dev32<4>>, g, b, 0, s, descs, ctrls, blocks, remap);
    }
    return hipGetLastError();
}

hipError_t launch_prime(int dim, int prec, const InstDesc* descs, InstCtrl* ctrls,
                        const BlockRef* blocks, int64_t nblocks, int waves, hipStream_t s)
{
    if (!grid_ok(nblocks) || waves < 1 || waves > 4) return hipErrorInvalidValue;
    dim3 g((unsigned)nblocks), b((unsigned)(64 * waves));
    if (dim == 2) {
        if (prec == 0)
            hipLaunchKernelGGL((prime_kernel<Plain64<5>, 5>), g, b, 0, s, descs, ctrls, blocks);
        else
            hipLaunchKernelGGL((prime_kernel<Dev32<5>, 5>), g, b, 0, s, descs, ctrls, blocks);
    } else {
        if (prec == 0)
            hipLaunchKernelGGL((prime_kernel<Plain64<4>, 4>), g, b, 0, s, descs, ctrls, blocks);
        else
            hipLaunchKernelGGL((prime_kernel<Dev32<4>, 4>), g, b, 0, s, descs, ctrls, blocks);
    }
    return hipGetLastError();
}

hipError_t launch_finalize(const InstDesc* descs, InstCtrl* ctrls, const int32_t* insts, int n,
                           int mode, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(finalize_kernel, dim3((unsigned)n), dim3(256), 0, s, descs, ctrls, insts,
                       mode);
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
