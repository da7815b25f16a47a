// ng_api.cpp -- the C ABI of include/ng.h: validation, device-memory layout
// inside the caller's buffer, batch bookkeeping, step sequencing (direct
// launches or captured HIP graphs) and state read-out.
//
// A single solve (ng_solver) is a batch of capacity one whose arena is exactly
// ng_state_bytes long, so one code path serves both.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <string>
#include <thread>
#include <utility>
#include <vector>

#include "../../include/ng.h"
#include "ng_internal.hpp"
#include "ng_launch.hpp"

using namespace ng;

namespace {

constexpr size_t kAlign = 256;
constexpr int kMinRows2D = 4;        // smallest rows-per-item the partial space allows
// rows (2D) or segments (1D) per item -1: chosen from the grids (auto_rows),
// the default
constexpr int kAutoRows = -1;
constexpr int kDefaultRows2D = kAutoRows;
constexpr int kDefaultSegs1D = kAutoRows;
// work items (one wavefront each) a solve's automatic shape aims for.  2D:
// about three quarters of the 3072 wavefronts the FP32 step kernel keeps
// resident (3 per SIMD); the 4096^2 grid has 8832 at 32 rows, smaller grids
// shorten their row chunks rather than leave SIMDs idle (256^2 FP32: 41 -> 15
// us per step at 4 rows, 1024^2: 43 -> 29 at 8, 2048^2: 84 -> 64 at 24).  1D: a lone 2^20-cell grid is fastest at
// 4 segments per item (4370 items), 2^17 at 2, 2^15 at 1 (FP64 2^15: 36 -> 17
// us per step against 8); 8 segments only pay with far more work, as in the
// 512-solve batch (16500 items: 4 segments cost it 9 %).
constexpr int64_t kAutoItems2D = 2304;
constexpr int kAutoRows2D[] = {32, 24, 16, 12, 8, 6, 4};
constexpr int64_t kAutoItems1D = 1024;
constexpr int64_t kAutoItems1DWide = 8192;   // for 8 segments per item
// waves per workgroup -1: 4, except 2 for 1D launches of fewer than
// kAutoItems1DWaves work items (FP64 2^15 cells: 17 -> 15 us per step)
constexpr int kDefaultWaves2D = 4;
constexpr int kDefaultWaves1D = kAutoRows;
constexpr int64_t kAutoItems1DWaves = 2048;
constexpr int kDefaultGraphSteps = 64;
// Solves up to this many cells run in the persistent one-workgroup kernel
// (many steps per launch); larger ones take one launch per step over the
// whole GPU.  Per-cell arithmetic is the same on both paths.
constexpr int64_t kSmallCells32 = 4096;
constexpr int64_t kSmallCells64 = 2048;
constexpr int kSmallRows2D = 8;
constexpr int kSmallSegs1D = 1;
constexpr int kSmallWaves = 8;
// Big solves of at most this many workgroups accept their steps inside the
// step kernel (last workgroup); beyond it the per-workgroup release fence costs
// more than the separate finalize launch.
constexpr int64_t kFusedMaxBlocks = 256;
// A batch's only solve, when it is 1D with at most this many cells and no
// forced source, runs in the cooperative kernel: many steps per launch over
// many workgroups, with a grid barrier per step instead of two launches.
constexpr int64_t kCoopCells = int64_t(1) << 22;
// polls of a grid-barrier wait before it gives up (each a memory round trip
// of about a microsecond and a short sleep: about a second)
constexpr int32_t kCoopSpin = 1 << 20;
// a cooperative launch gives each work item a wave of its own, four waves
// per workgroup (one per SIMD of a CU), while the items fit in that many
// workgroups; more items take the kernel's largest workgroups
constexpr int kCoopSmallWaves = 4;
// Pinned staging buffers of the initial-state upload (two, used in turn).
constexpr size_t kStageBytes = size_t(16) << 20;
// Host threads converting one staging chunk, and the cells each takes at least.
constexpr int kHostThreads = 8;
constexpr int64_t kCellsPerThread = 65536;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

int ncomp(int ndim) { return ndim == 2 ? 5 : 4; }
size_t real_size(int prec) { return prec == NG_FP32 ? 4 : 8; }
bool prec_ok(int prec) { return prec == NG_FP32 || prec == NG_FP64 || prec == NG_MIXED; }
// kernel family of a precision: FP64 throughout, FP32 deviations, FP32
// arithmetic on FP64 deviations
int kind_of(int prec) { return prec == NG_FP64 ? 0 : (prec == NG_FP32 ? 1 : 2); }

// strips (2D) or segments (1D) of a grid; 1D counts the shorter segments of
// the CSPH-TVD step, the most either scheme gives
int64_t strips_of(const ng_grid* g) { return cdiv(g->nx, g->ndim == 2 ? kInterior : kCsphInterior); }

// most workgroups any allowed launch shape gives this grid (1 wave per block,
// smallest rows per item)
int64_t partial_cap_of(const ng_grid* g)
{
    if (g->ndim == 2) return strips_of(g) * cdiv(g->ny, kMinRows2D);
    return strips_of(g);
}

size_t state_plane_bytes(const ng_grid* g, int prec)
{
    return align_up((size_t)(g->nx * g->ny) * ncomp(g->ndim) * real_size(prec));
}

size_t solve_bytes(const ng_grid* g, int prec)
{
    return 2 * state_plane_bytes(g, prec) + align_up((size_t)partial_cap_of(g) * sizeof(Partial));
}

struct Layout {
    size_t descs, ctrls, insts, iota, coop, blocks1, blocks2, heap;
};

Layout header_layout(int capacity, size_t tcap1, size_t tcap2)
{
    Layout L;
    size_t o = 0;
    L.descs = o;
    o += align_up(sizeof(InstDesc) * capacity);
    L.ctrls = o;
    o += align_up(sizeof(InstCtrl) * capacity);
    L.insts = o;
    o += align_up(sizeof(int32_t) * 5 * capacity);
    L.iota = o;
    o += align_up(sizeof(int32_t) * capacity);
    L.coop = o;
    o += align_up(sizeof(CoopSync));
    L.blocks1 = o;
    o += align_up(sizeof(BlockRef) * tcap1);
    L.blocks2 = o;
    o += align_up(sizeof(BlockRef) * tcap2);
    L.heap = o;
    return L;
}

bool finite_pos(double x) { return isfinite(x) && x > 0.0; }

int validate(const ng_gas* gas, const ng_grid* grid, const ng_numerics* num, std::string& err)
{
    if (!gas || !grid || !num) {
        err = "null argument";
        return NG_EINVAL;
    }
    const double gv[] = {gas->gamma, gas->R, gas->Cv, gas->rho0, gas->T0, gas->tau0,
                         gas->tau_rho, gas->tau_T, gas->Q0, gas->Q_rho, gas->Q_T, gas->I0,
                         gas->I_rho, gas->I_T, gas->fx, gas->fy};
    for (double x : gv)
        if (!isfinite(x)) {
            err = "non-finite gas parameter";
            return NG_EINVAL;
        }
    if (!(gas->gamma > 1.0)) { err = "gamma must exceed 1"; return NG_EINVAL; }
    if (!(gas->R > 0.0)) { err = "R must be positive"; return NG_EINVAL; }
    if (!(gas->Cv >= 0.0)) { err = "Cv must be non-negative"; return NG_EINVAL; }
    if (!(gas->rho0 > 0.0) || !(gas->T0 > 0.0)) { err = "rho0 and T0 must be positive"; return NG_EINVAL; }
    if (!(gas->tau0 > 0.0)) { err = "tau0 must be positive"; return NG_EINVAL; }
    if (!(gas->Q0 >= 0.0) || !(gas->I0 >= 0.0)) { err = "Q0 and I0 must be non-negative"; return NG_EINVAL; }
    if (grid->ndim != 1 && grid->ndim != 2) { err = "ndim must be 1 or 2"; return NG_EINVAL; }
    if (grid->nx < 4 || (grid->ndim == 2 && grid->ny < 4) || (grid->ndim == 1 && grid->ny != 1)) {
        err = "need nx >= 4 (and ny >= 4 in 2D, ny == 1 in 1D)";
        return NG_EINVAL;
    }
    if (grid->nx > (1LL << 31) || grid->ny > (1LL << 31) || grid->nx * grid->ny > (1LL << 33)) {
        err = "grid too large";
        return NG_EINVAL;
    }
    if (!finite_pos(grid->h)) { err = "h must be positive"; return NG_EINVAL; }
    for (int i = 0; i < (grid->ndim == 2 ? 4 : 2); i++)
        if (grid->bc[i] != NG_BC_PERIODIC && grid->bc[i] != NG_BC_WALL &&
            grid->bc[i] != NG_BC_OUTFLOW && !(i == 0 && grid->bc[i] == NG_BC_SOURCE)) {
            err = "unknown boundary kind (a source is allowed at the x-low end only)";
            return NG_EINVAL;
        }
    if (grid->bc[0] == NG_BC_SOURCE &&
        (!finite_pos(grid->src_lambda) || !isfinite(grid->src_amp) ||
         !(fabs(grid->src_amp) < 0.5 * gas->rho0))) {
        err = "source needs src_lambda > 0 and |src_amp| < rho0 / 2";
        return NG_EINVAL;
    }
    if (grid->bc[0] == NG_BC_SOURCE && grid->src_hw > 0.0 &&
        (grid->ndim != 2 || !isfinite(grid->src_yc) || !isfinite(grid->src_hw))) {
        err = "a source segment needs a 2D grid and finite src_yc, src_hw";
        return NG_EINVAL;
    }
    if (!isfinite(grid->wedge_tan) ||
        (grid->wedge_tan > 0.0 && (grid->ndim != 2 || !(grid->wedge_x0 >= 0.0) ||
                                   !isfinite(grid->wedge_x0) || !isfinite(grid->wedge_y0)))) {
        err = "an active wedge needs a 2D grid, finite wedge_y0 and 0 <= wedge_x0 < inf";
        return NG_EINVAL;
    }
    for (int a = 0; a < 2; a++)
        if ((grid->bc[2 * a] == NG_BC_PERIODIC) != (grid->bc[2 * a + 1] == NG_BC_PERIODIC) &&
            (a == 0 || grid->ndim == 2)) {
            err = "a periodic axis needs both ends periodic";
            return NG_EINVAL;
        }
    if (prec_ok(num->precision)) {
        const uint64_t cells = (uint64_t)grid->nx * (uint64_t)(grid->ndim == 2 ? grid->ny : 1);
        if (cells * real_size(num->precision) > (1ULL << 32)) {
            err = "grid too large for 32-bit plane offsets";
            return NG_EINVAL;
        }
    }
    if (grid->ndim == 1 && gas->fy != 0.0) { err = "fy must be 0 in 1D"; return NG_EINVAL; }
    if (!(num->cfl > 0.0 && num->cfl < 1.0)) { err = "cfl must lie in (0, 1)"; return NG_EINVAL; }
    if (num->riemann != NG_HLLC && num->riemann != NG_HLL) { err = "unknown riemann solver"; return NG_EINVAL; }
    if (num->limiter != NG_MINMOD) { err = "unknown limiter"; return NG_EINVAL; }
    if (!prec_ok(num->precision)) { err = "unknown precision"; return NG_EINVAL; }
    if (!(num->stiff_z >= 0.0)) { err = "stiff_z must be >= 0"; return NG_EINVAL; }
    if (num->scheme != NG_MUSCL && num->scheme != NG_CSPH_TVD) { err = "unknown scheme"; return NG_EINVAL; }
    if (num->scheme == NG_CSPH_TVD &&
        (grid->ndim != 1 || num->precision != NG_FP64 || num->riemann != NG_HLL)) {
        err = "the CSPH-TVD step needs a 1D grid, NG_FP64 and NG_HLL";
        return NG_EINVAL;
    }
    return NG_OK;
}

// E = p/(gamma-1) + rho |v|^2 / 2 + E_nu  (eq. (5)); host-side conversions
void prim_to_cons_cell(double gm1, int nc, const double* W, double* U)
{
    if (nc == 5) {
        double rho = W[0], u = W[1], v = W[2], p = W[3], e = W[4];
        U[0] = rho;
        U[1] = rho * u;
        U[2] = rho * v;
        U[3] = p / gm1 + 0.5 * rho * (u * u + v * v) + e;
        U[4] = e;
    } else {
        double rho = W[0], u = W[1], p = W[2], e = W[3];
        U[0] = rho;
        U[1] = rho * u;
        U[2] = p / gm1 + 0.5 * rho * (u * u) + e;
        U[3] = e;
    }
}

void cons_to_prim_cell(double gm1, int nc, const double* U, double* W)
{
    double rho = U[0];
    double u = U[1] / rho;
    if (nc == 5) {
        double v = U[2] / rho;
        double ke = 0.5 * rho * (u * u + v * v);
        W[0] = rho;
        W[1] = u;
        W[2] = v;
        W[3] = gm1 * (U[3] - ke - U[4]);
        W[4] = U[4];
    } else {
        double ke = 0.5 * rho * (u * u);
        W[0] = rho;
        W[1] = u;
        W[2] = gm1 * (U[2] - ke - U[3]);
        W[3] = U[3];
    }
}

struct Slot {
    bool live = false;
    int dim = 0;
    InstDesc d{};
    size_t off = 0, bytes = 0;
    int64_t partial_cap = 0;
    int64_t block_off = 0;  // first entry in the dim's block table
    int pos = 0;            // index in the dim's instance list (big or small)
    bool small = false;     // advanced by the persistent one-workgroup kernel
    bool coop = false;      // advanced by the cooperative kernel
    bool reported = false;
};

}  // namespace

struct ng_batch {
    int capacity = 0;
    int prec = 0;
    char* arena = nullptr;
    size_t arena_bytes = 0;
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;
    Layout L{};
    size_t tcap[3] = {0, 0, 0};
    std::vector<Slot> slots;
    std::map<size_t, size_t> free_list;  // offset -> size
    int rows[3] = {0, kDefaultSegs1D, kDefaultRows2D};
    int auto_rows[3] = {0, 0, 0};   // automatic shape of the current big solves
    int waves[3] = {0, kDefaultWaves1D, kDefaultWaves2D};
    int auto_waves[3] = {0, 0, 0};  // automatic waves per workgroup of the big solves
    int remap = 1;
    int64_t small_limit = -1;  // cells; -1: by precision, 0: persistent path off
    int64_t coop_limit = -1;   // cells; -1: kCoopCells, 0: cooperative path off
    int32_t coop_spin = kCoopSpin;
    int coop_slot = -1;        // the solve the cooperative kernel advances, or -1
    int coop_grid = 0, coop_waves = 0, coop_variant = 0;
    int dev_coop = -1;         // cooperative launch supported (-1: not asked yet)
    int dev_cus = 0;
    int fused = 1;             // step kernels accept their own step (last workgroup)
    int64_t nblocks[3] = {0, 0, 0};   // workgroups of the per-step launch (big solves)
    int ninst[3] = {0, 0, 0};         // big solves per dim
    int nsep[3] = {0, 0, 0};          // big solves accepted by the finalize kernel
    int variant[3] = {0, 0, 0};       // step kernel variant of the per-step launch
    int nsmall[3] = {0, 0, 0};        // small solves per dim
    bool dirty = true;
    // captured step sequence
    hipGraphExec_t gexec = nullptr;
    int gsteps = 0;
    int graph_steps = kDefaultGraphSteps;
    // pinned read-back of the control blocks
    InstCtrl* h_ctrls = nullptr;
    // initial-state uploads run on a second stream, so that admitting a solve
    // overlaps the steps in flight: chunks are converted into two pinned
    // staging buffers in turn; descriptor and control block go through pinned
    // per-slot copies; ev_ready marks the end of the last upload
    hipStream_t up_stream = nullptr;
    void* stage[2] = {nullptr, nullptr};
    size_t stage_bytes = 0;
    hipEvent_t ev_stage[2] = {nullptr, nullptr};
    hipEvent_t ev_ready = nullptr;
    InstDesc* h_desc_up = nullptr;
    InstCtrl* h_ctrl_up = nullptr;
    std::vector<BlockRef> h_blocks[3];
    std::vector<int32_t> h_insts;
    // timing
    bool timing = false;
    int timing_every = 1;
    std::vector<hipEvent_t> ev_pool;
    double t_step_ms = 0.0, t_fin_ms = 0.0;
    int64_t t_launches = 0;
    std::string err;

    InstDesc* d_descs() { return (InstDesc*)(arena + L.descs); }
    InstCtrl* d_ctrls() { return (InstCtrl*)(arena + L.ctrls); }
    int32_t* d_insts(int dim) { return (int32_t*)(arena + L.insts) + dim * capacity; }
    int32_t* d_small(int dim) { return (int32_t*)(arena + L.insts) + (2 + dim) * capacity; }
    int32_t* d_iota() { return (int32_t*)(arena + L.iota); }
    CoopSync* d_coop() { return (CoopSync*)(arena + L.coop); }
    BlockRef* d_blocks(int dim) { return (BlockRef*)(arena + (dim == 1 ? L.blocks1 : L.blocks2)); }
};

struct ng_solver {
    ng_batch* b = nullptr;
    int slot = 0;
    std::string err;
};

static_assert(NG_ESTALL == ng::kStatusStall, "status of a stalled cooperative launch");
static_assert(NG_MUSCL == ng::kSchemeMuscl && NG_CSPH_TVD == ng::kSchemeCsph,
              "schemes of the ABI and the kernels");
static_assert(NG_BC_PERIODIC == ng::kBcPeriodic && NG_BC_WALL == ng::kBcWall &&
                  NG_BC_OUTFLOW == ng::kBcOutflow && NG_BC_SOURCE == ng::kBcSource,
              "boundary kinds of the ABI and the kernels");

namespace {

int dev_err(ng_batch* b, hipError_t e, const char* what)
{
    b->err = std::string(what) + ": " + hipGetErrorString(e);
    return NG_EDEVICE;
}
#define CK(b, call)                                         \
    do {                                                    \
        hipError_t e_ = (call);                             \
        if (e_ != hipSuccess) return dev_err((b), e_, #call); \
    } while (0)

// Destroy the captured step sequence; launches of it may still be in flight
// on the batch stream (ng_set_graph_steps, a new length in ensure_graph), so
// the stream is drained first.
void drop_graph(ng_batch* b)
{
    if (b->gexec) {
        (void)hipStreamSynchronize(b->stream);
        (void)hipGraphExecDestroy(b->gexec);
        b->gexec = nullptr;
    }
    b->gsteps = 0;
}

bool arena_alloc(ng_batch* b, size_t bytes, size_t* off)
{
    for (auto it = b->free_list.begin(); it != b->free_list.end(); ++it) {
        if (it->second >= bytes) {
            *off = it->first;
            size_t rest = it->second - bytes;
            size_t noff = it->first + bytes;
            b->free_list.erase(it);
            if (rest) b->free_list[noff] = rest;
            return true;
        }
    }
    return false;
}

void arena_free(ng_batch* b, size_t off, size_t bytes)
{
    auto it = b->free_list.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != b->free_list.end() && it->first + it->second == nx->first) {
        it->second += nx->second;
        b->free_list.erase(nx);
    }
    if (it != b->free_list.begin()) {
        auto pv = std::prev(it);
        if (pv->first + pv->second == it->first) {
            pv->second += it->second;
            b->free_list.erase(it);
        }
    }
}

// A free slot and a free arena block of `bytes` exist.
bool has_room(const ng_batch* b, size_t bytes)
{
    bool slot = false;
    for (int i = 0; i < b->capacity && !slot; i++) slot = !b->slots[i].live;
    if (!slot) return false;
    for (const auto& kv : b->free_list)
        if (kv.second >= bytes) return true;
    return false;
}

// Work items of a grid at r rows (2D) or r segments (1D) per item.
int64_t items_at(int dim, int64_t nx, int64_t ny, int r)
{
    const int64_t strips = cdiv(nx, kInterior);
    return dim == 2 ? strips * cdiv(ny, r) : cdiv(strips, r);
}

// Rows (2D) or 60-cell segments (1D) per work item under the automatic shape,
// one value for all big solves of a dim launched together (grids given as
// (nx, ny) pairs): 2D the largest of kAutoRows2D at which their work items
// add up to kAutoItems2D, else 4; 1D 8 segments if they give
// kAutoItems1DWide items, else the largest of 4, 2 and 1 reaching
// kAutoItems1D, else 1.  A batch with work enough for the whole GPU
// keeps long chunks (fewer halo rows); a lone small grid gets short ones.
int auto_rows(int dim, const std::vector<std::pair<int64_t, int64_t>>& grids)
{
    auto items = [&](int r) {
        int64_t n = 0;
        for (const auto& g : grids) n += items_at(dim, g.first, g.second, r);
        return n;
    };
    if (dim == 2) {
        for (int r : kAutoRows2D)
            if (items(r) >= kAutoItems2D) return r;
        return kMinRows2D;
    }
    if (items(8) >= kAutoItems1DWide) return 8;
    for (int r = 4; r > 1; r >>= 1)
        if (items(r) >= kAutoItems1D) return r;
    return 1;
}

// Waves per workgroup of a dim's big-solve launch: the set value, else the
// automatic one of the current solves, else (a solve not yet in the tables)
// that of the given grids alone.
int waves_of(const ng_batch* b, int dim, const std::vector<std::pair<int64_t, int64_t>>& grids)
{
    if (b->waves[dim] > 0) return b->waves[dim];
    if (b->auto_waves[dim] > 0) return b->auto_waves[dim];
    if (dim == 2) return kDefaultWaves2D;
    const int r = b->rows[1] > 0 ? b->rows[1] : auto_rows(1, grids);
    int64_t n = 0;
    for (const auto& g : grids) n += items_at(1, g.first, g.second, r);
    return n < kAutoItems1DWaves ? 2 : 4;
}

// Work decomposition of one solve for the current launch shape of its dim.
// A solve accepts its own steps inside the step kernel only when it is the one
// big solve of its dim: with several, each of their workgroups would pay the
// release fence, which costs more than one finalize launch for all of them.
void shape_solve(ng_batch* b, Slot& s, bool alone = true)
{
    InstDesc& d = s.d;
    int dim = s.dim;
    d.waves_per_block = s.small ? 1 : (s.coop ? kCoopSmallWaves : waves_of(b, dim, {{d.nx, d.ny}}));
    if (s.small)
        d.rows_per_item = dim == 2 ? kSmallRows2D : kSmallSegs1D;
    else if (s.coop)
        d.rows_per_item = 1;
    else if (b->rows[dim] != kAutoRows)
        d.rows_per_item = b->rows[dim];
    else if (b->auto_rows[dim] > 0)
        d.rows_per_item = b->auto_rows[dim];
    else
        d.rows_per_item = auto_rows(dim, {{d.nx, d.ny}});
    d.nstrips = (int32_t)cdiv(d.nx, dim == 2 ? kInterior : seg_cells(d.scheme));
    if (dim == 2)
        d.nchunks = (int32_t)cdiv(d.ny, d.rows_per_item);
    else
        d.nchunks = (int32_t)cdiv(d.nstrips, d.rows_per_item);
    d.nitems = dim == 2 ? (int64_t)d.nstrips * d.nchunks : (int64_t)d.nchunks;
    d.nblocks = cdiv(d.nitems, d.waves_per_block);
    d.fused = (b->fused && alone && !s.small && d.nblocks <= kFusedMaxBlocks) ? 1 : 0;
}

// The cooperative path: a batch whose only live solve is 1D, has no forced
// source and at most coop_limit cells, on a device that supports cooperative
// launches.  Marks that solve (Slot::coop), sets coop_slot (else -1) and the
// launch shape: while the segments (60 cells, 58 for CSPH-TVD) fit one per
// wave in workgroups of kCoopSmallWaves waves (one per SIMD) with at most one
// workgroup per CU, that; else workgroups of the kernel's largest size, as
// many as stay resident together (and have a segment for every wave), at
// most kCoopFlat (the slots of the grid barrier); the kernel deals the
// segments to the waves in runs.
int choose_coop(ng_batch* b)
{
    b->coop_slot = -1;
    int live = 0, cand = -1;
    for (int i = 0; i < b->capacity; i++) {
        Slot& s = b->slots[i];
        s.coop = false;
        if (!s.live) continue;
        live++;
        cand = i;
    }
    const int64_t lim = b->coop_limit >= 0 ? b->coop_limit : kCoopCells;
    if (live != 1 || lim == 0) return NG_OK;
    Slot& s = b->slots[cand];
    if (s.dim != 1 || s.d.ncell > lim) return NG_OK;
    if (b->dev_coop < 0) {
        int dev = 0, coop = 0, cus = 0;
        CK(b, hipGetDevice(&dev));
        CK(b, hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
        CK(b, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        b->dev_coop = coop ? 1 : 0;
        b->dev_cus = cus;
    }
    if (!b->dev_coop || b->dev_cus < 1) return NG_OK;
    const int kind = kind_of(b->prec);
    const int v = s.d.scheme == kSchemeCsph
                      ? kVariantCsph
                      : ((s.d.riemann == NG_HLLC && !s.d.any_bc) ? 1 + s.d.cl_recipe : 0);
    const int64_t segs = cdiv(s.d.nx, seg_cells(s.d.scheme));
    int per_cu = 0, maxw = 0;
    CK(b, coop_capacity(kind, v, kCoopSmallWaves, &per_cu, &maxw));
    int waves = kCoopSmallWaves;
    if (segs > (int64_t)kCoopSmallWaves * b->dev_cus) {
        waves = maxw;
        CK(b, coop_capacity(kind, v, waves, &per_cu, &maxw));
    }
    const int64_t resident = (int64_t)per_cu * b->dev_cus;
    const int64_t grid = std::min<int64_t>(std::min<int64_t>(cdiv(segs, waves), resident),
                                           kCoopFlat);
    if (grid < 1 || coop_space((uint64_t)grid) > (uint64_t)s.partial_cap * sizeof(Partial))
        return NG_OK;
    s.coop = true;
    b->coop_slot = cand;
    b->coop_grid = (int)grid;
    b->coop_waves = waves;
    b->coop_variant = v;
    return NG_OK;
}

// Launch the cooperative kernel for nsteps steps (in launches of at most
// kCoopMaxSteps steps).
int enqueue_coop(ng_batch* b, int64_t nsteps)
{
    for (int64_t left = nsteps; left > 0;) {
        const int64_t n = std::min<int64_t>(left, kCoopMaxSteps);
        CK(b, launch_coop(kind_of(b->prec), b->coop_variant, b->d_descs(), b->d_ctrls(),
                          b->coop_slot, b->d_coop(), b->coop_grid, b->coop_waves, n,
                          b->coop_spin, b->stream));
        left -= n;
    }
    return NG_OK;
}

// Rebuild the device tables (descriptors, per-dim solve lists and workgroup
// maps) after the set of solves or a launch shape changed.  Synchronising.
int rebuild(ng_batch* b)
{
    if (!b->dirty) return NG_OK;
    std::vector<int32_t> insts(5 * b->capacity, 0);
    for (int dim = 1; dim <= 2; dim++) {
        b->h_blocks[dim].clear();
        b->ninst[dim] = 0;
        b->nsep[dim] = 0;
        b->nsmall[dim] = 0;
    }
    // per dim: the workgroups of big solves first (the per-step launch covers
    // exactly those), then those of small solves (used by the priming pass only)
    const int64_t lim = b->small_limit >= 0 ? b->small_limit
                                            : (b->prec != NG_FP64 ? kSmallCells32 : kSmallCells64);
    int rc = choose_coop(b);
    if (rc) return rc;
    int nbig[3] = {0, 0, 0};
    std::vector<std::pair<int64_t, int64_t>> grids[3];
    for (int i = 0; i < b->capacity; i++)
        if (b->slots[i].live) {
            Slot& s = b->slots[i];
            s.small = !s.coop && s.d.ncell <= lim;
            if (!s.small) {
                nbig[s.dim]++;
                grids[s.dim].push_back({s.d.nx, s.d.ny});
            }
        }
    for (int dim = 1; dim <= 2; dim++) {
        b->auto_rows[dim] = 0;
        b->auto_waves[dim] = 0;
        if (grids[dim].empty()) continue;
        b->auto_rows[dim] = auto_rows(dim, grids[dim]);
        b->auto_waves[dim] = waves_of(b, dim, grids[dim]);
    }
    for (int pass = 0; pass < 2; pass++) {
        for (int i = 0; i < b->capacity; i++) {
            Slot& s = b->slots[i];
            if (!s.live || (int)s.small != pass) continue;
            shape_solve(b, s, nbig[s.dim] <= 1);
            if (s.d.nblocks > s.partial_cap) {
                b->err = "launch shape needs more reduction records than reserved";
                return NG_EINVAL;
            }
            auto& tab = b->h_blocks[s.dim];
            s.block_off = (int64_t)tab.size();
            for (int64_t j = 0; j < s.d.nblocks; j++) tab.push_back(BlockRef{i, (int32_t)j});
            if (s.small) {
                s.pos = b->nsmall[s.dim]++;
                insts[(2 + s.dim) * b->capacity + s.pos] = i;
            } else {
                s.pos = b->ninst[s.dim]++;
                insts[s.dim * b->capacity + s.pos] = i;
                b->nblocks[s.dim] = (int64_t)tab.size();
                if (!s.d.fused) b->nsep[s.dim]++;
            }
        }
    }
    // the step kernel variant of each dim's launch: the periodic-HLLC kernel
    // of a closure recipe when every big solve has that path, else the general
    for (int dim = 1; dim <= 2; dim++) {
        int v = -1;
        for (int i = 0; i < b->capacity; i++) {
            const Slot& s = b->slots[i];
            if (!s.live || s.small || s.dim != dim) continue;
            const int sv = s.d.scheme == kSchemeCsph
                               ? kVariantCsph
                               : ((s.d.riemann == NG_HLLC && !s.d.any_bc) ? 1 + s.d.cl_recipe : 0);
            v = (v < 0 || v == sv) ? sv : 0;
        }
        b->variant[dim] = v < 0 ? 0 : v;
    }
    for (int dim = 1; dim <= 2; dim++) {
        if (b->h_blocks[dim].size() > b->tcap[dim]) {
            b->err = "workgroup table capacity exceeded";
            return NG_ENOMEM;
        }
        if (!b->ninst[dim]) b->nblocks[dim] = 0;
    }
    std::vector<InstDesc> descs(b->capacity);
    for (int i = 0; i < b->capacity; i++) descs[i] = b->slots[i].d;
    CK(b, hipMemcpyAsync(b->d_descs(), descs.data(), sizeof(InstDesc) * b->capacity,
                         hipMemcpyHostToDevice, b->stream));
    CK(b, hipMemcpyAsync(b->arena + b->L.insts, insts.data(), sizeof(int32_t) * insts.size(),
                         hipMemcpyHostToDevice, b->stream));
    for (int dim = 1; dim <= 2; dim++)
        if (!b->h_blocks[dim].empty())
            CK(b, hipMemcpyAsync(b->d_blocks(dim), b->h_blocks[dim].data(),
                                 sizeof(BlockRef) * b->h_blocks[dim].size(),
                                 hipMemcpyHostToDevice, b->stream));
    CK(b, hipStreamSynchronize(b->stream));
    drop_graph(b);
    b->dirty = false;
    return NG_OK;
}

hipEvent_t get_event(ng_batch* b, size_t i)
{
    while (b->ev_pool.size() <= i) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        b->ev_pool.push_back(e);
    }
    return b->ev_pool[i];
}

// Enqueue the kernels of one step of every active solve on stream st.
int enqueue_one(ng_batch* b, hipStream_t st)
{
    for (int dim = 1; dim <= 2; dim++) {
        if (!b->ninst[dim]) continue;
        CK(b, launch_step(dim, kind_of(b->prec), b->variant[dim], b->d_descs(), b->d_ctrls(),
                          b->d_blocks(dim), b->nblocks[dim], waves_of(b, dim, {}), b->remap, b->fused,
                          st));
        if (b->nsep[dim])
            CK(b, launch_finalize(b->d_descs(), b->d_ctrls(), b->d_insts(dim), b->ninst[dim], 0,
                                  st));
    }
    return NG_OK;
}

// Launch the persistent kernel of the small solves for nsteps steps.
int enqueue_small(ng_batch* b, int64_t nsteps, hipStream_t st)
{
    for (int dim = 1; dim <= 2; dim++) {
        if (!b->nsmall[dim]) continue;
        CK(b, launch_small(dim, kind_of(b->prec), b->d_descs(), b->d_ctrls(),
                           b->d_small(dim), b->nsmall[dim], kSmallWaves, nsteps, st));
    }
    return NG_OK;
}

bool any_big(const ng_batch* b) { return b->ninst[1] + b->ninst[2] > 0; }
bool any_small(const ng_batch* b) { return b->nsmall[1] + b->nsmall[2] > 0; }

// Timed variant: the step and finalize kernels (big solves) of every
// timing_every-th step and of the last step record their own start and end in
// events of the pool (no event packets between launches), the other steps
// launch as in enqueue_one;
// small solves: events around the persistent launch (reported per step).
int enqueue_timed(ng_batch* b, int64_t nsteps)
{
    size_t ne = 0;
    std::vector<std::pair<size_t, size_t>> step_pairs, fin_pairs;
    double small_ms = 0.0;
    if (b->coop_slot >= 0) {
        hipEvent_t e0 = get_event(b, 0), e1 = get_event(b, 1);
        if (!e0 || !e1) return dev_err(b, hipErrorOutOfMemory, "hipEventCreate");
        CK(b, hipEventRecord(e0, b->stream));
        int rc = enqueue_coop(b, nsteps);
        if (rc) return rc;
        CK(b, hipEventRecord(e1, b->stream));
        CK(b, hipStreamSynchronize(b->stream));
        float ms = 0.f;
        CK(b, hipEventElapsedTime(&ms, e0, e1));
        b->t_step_ms = nsteps > 0 ? ms / nsteps : 0.0;
        b->t_fin_ms = 0.0;
        b->t_launches = cdiv(nsteps, kCoopMaxSteps);
        return NG_OK;
    }
    if (any_small(b)) {
        hipEvent_t e0 = get_event(b, 0), e1 = get_event(b, 1);
        if (!e0 || !e1) return dev_err(b, hipErrorOutOfMemory, "hipEventCreate");
        CK(b, hipEventRecord(e0, b->stream));
        int rc = enqueue_small(b, nsteps, b->stream);
        if (rc) return rc;
        CK(b, hipEventRecord(e1, b->stream));
        CK(b, hipStreamSynchronize(b->stream));
        float ms = 0.f;
        CK(b, hipEventElapsedTime(&ms, e0, e1));
        small_ms = ms;
        ne = 2;
    }
    for (int64_t i = 0; i < nsteps && any_big(b); i++) {
        // time steps every-1, 2*every-1, ... and the last one: the first timed
        // launch never follows an idle GPU
        if ((i + 1) % b->timing_every && i != nsteps - 1) {
            int rc = enqueue_one(b, b->stream);
            if (rc) return rc;
            continue;
        }
        for (int dim = 1; dim <= 2; dim++) {
            if (!b->ninst[dim]) continue;
            hipEvent_t e0 = get_event(b, ne), e1 = get_event(b, ne + 1), e2 = get_event(b, ne + 2),
                       e3 = get_event(b, ne + 3);
            if (!e0 || !e1 || !e2 || !e3) return dev_err(b, hipErrorOutOfMemory, "hipEventCreate");
            CK(b, launch_step(dim, kind_of(b->prec), b->variant[dim], b->d_descs(), b->d_ctrls(),
                              b->d_blocks(dim), b->nblocks[dim], waves_of(b, dim, {}), b->remap,
                              b->fused, b->stream, e0, e1));
            step_pairs.push_back({ne, ne + 1});
            if (b->nsep[dim]) {
                CK(b, launch_finalize(b->d_descs(), b->d_ctrls(), b->d_insts(dim), b->ninst[dim],
                                      0, b->stream, e2, e3));
                fin_pairs.push_back({ne + 2, ne + 3});
            }
            ne += 4;
        }
    }
    CK(b, hipStreamSynchronize(b->stream));
    double ts = 0.0, tf = 0.0;
    for (auto& p : step_pairs) {
        float ms = 0.f;
        CK(b, hipEventElapsedTime(&ms, b->ev_pool[p.first], b->ev_pool[p.second]));
        ts += ms;
    }
    for (auto& p : fin_pairs) {
        float ms = 0.f;
        CK(b, hipEventElapsedTime(&ms, b->ev_pool[p.first], b->ev_pool[p.second]));
        tf += ms;
    }
    if (!step_pairs.empty()) {
        b->t_step_ms = ts / step_pairs.size();
        b->t_fin_ms = fin_pairs.empty() ? 0.0 : tf / fin_pairs.size();
        b->t_launches = (int64_t)step_pairs.size();
    } else {
        b->t_step_ms = nsteps > 0 ? small_ms / nsteps : 0.0;
        b->t_fin_ms = 0.0;
        b->t_launches = any_small(b) ? 1 : 0;
    }
    return NG_OK;
}

int ensure_graph(ng_batch* b)
{
    if (b->gexec && b->gsteps == b->graph_steps) return NG_OK;
    drop_graph(b);
    if (!b->cap_stream) CK(b, hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
    CK(b, hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
    int rc = NG_OK;
    for (int i = 0; i < b->graph_steps && rc == NG_OK; i++) rc = enqueue_one(b, b->cap_stream);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
    if (rc != NG_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return dev_err(b, e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        b->gexec = nullptr;
        return dev_err(b, e, "hipGraphInstantiate");
    }
    b->gsteps = b->graph_steps;
    return NG_OK;
}

// Enqueue nsteps steps: the cooperative solve in cooperative launches; else
// the small solves in one persistent launch, the big ones as whole captured
// graphs, then single launches for the rest.
int enqueue_steps(ng_batch* b, int64_t nsteps)
{
    int rc = rebuild(b);
    if (rc) return rc;
    if (b->timing) return enqueue_timed(b, nsteps);
    if (b->coop_slot >= 0) return enqueue_coop(b, nsteps);
    rc = enqueue_small(b, nsteps, b->stream);
    if (rc || !any_big(b)) return rc;
    int64_t left = nsteps;
    if (left >= b->graph_steps) {
        rc = ensure_graph(b);
        if (rc) return rc;
        while (left >= b->gsteps) {
            CK(b, hipGraphLaunch(b->gexec, b->stream));
            left -= b->gsteps;
        }
    }
    for (int64_t i = 0; i < left; i++) {
        rc = enqueue_one(b, b->stream);
        if (rc) return rc;
    }
    return NG_OK;
}

int read_ctrls(ng_batch* b)
{
    CK(b, hipMemcpyAsync(b->h_ctrls, b->d_ctrls(), sizeof(InstCtrl) * b->capacity,
                         hipMemcpyDeviceToHost, b->stream));
    CK(b, hipStreamSynchronize(b->stream));
    return NG_OK;
}

int set_limits(ng_batch* b, const std::vector<int32_t>& slots, double t_end, int64_t max_steps)
{
    if (slots.empty()) return NG_OK;
    // the instance list of a dim lives in device memory; use a scratch copy of
    // the requested slots in the unused third list
    int32_t* dl = b->d_insts(0);
    CK(b, hipMemcpyAsync(dl, slots.data(), sizeof(int32_t) * slots.size(), hipMemcpyHostToDevice,
                         b->stream));
    CK(b, launch_set_limits(b->d_ctrls(), dl, (int)slots.size(), t_end, max_steps, b->stream));
    CK(b, hipStreamSynchronize(b->stream));
    return NG_OK;
}

// Create the batch object over an arena (shared by ng_batch_create and the
// single-solve constructor).
int batch_new(int32_t capacity, int32_t precision, void* dev_buf, size_t dev_bytes,
              void* hip_stream, size_t tcap1, size_t tcap2, ng_batch** out, std::string& err)
{
    if (capacity < 1 || !dev_buf || !out || !prec_ok(precision)) {
        err = "invalid batch arguments";
        return NG_EINVAL;
    }
    if (((uintptr_t)dev_buf) % kAlign) {
        err = "device buffer must be 256-byte aligned";
        return NG_EINVAL;
    }
    Layout L = header_layout(capacity, tcap1, tcap2);
    if (dev_bytes < L.heap) {
        err = "device buffer too small for the batch header";
        return NG_ENOMEM;
    }
    ng_batch* b = new ng_batch();
    b->capacity = capacity;
    b->prec = precision;
    b->arena = (char*)dev_buf;
    b->arena_bytes = dev_bytes;
    b->stream = (hipStream_t)hip_stream;
    b->L = L;
    b->tcap[1] = tcap1;
    b->tcap[2] = tcap2;
    b->slots.resize(capacity);
    if (dev_bytes > L.heap) b->free_list[L.heap] = dev_bytes - L.heap;
    hipError_t e = hipHostMalloc((void**)&b->h_ctrls, sizeof(InstCtrl) * capacity, 0);
    if (e == hipSuccess) e = hipHostMalloc((void**)&b->h_desc_up, sizeof(InstDesc) * capacity, 0);
    if (e == hipSuccess) e = hipHostMalloc((void**)&b->h_ctrl_up, sizeof(InstCtrl) * capacity, 0);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->up_stream, hipStreamNonBlocking);
    for (int k = 0; k < 2 && e == hipSuccess; k++)
        e = hipEventCreateWithFlags(&b->ev_stage[k], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_ready, hipEventDisableTiming);
    // recorded once so that the first waits on them return at once
    for (int k = 0; k < 2 && e == hipSuccess; k++) e = hipEventRecord(b->ev_stage[k], b->up_stream);
    if (e == hipSuccess) e = hipEventRecord(b->ev_ready, b->up_stream);
    // zero the control blocks so that unused slots are inert; slot index list
    std::vector<InstCtrl> z(capacity);
    for (auto& c : z) {
        memset(&c, 0, sizeof(c));
        c.status = -1;
    }
    std::vector<int32_t> iota(capacity);
    for (int i = 0; i < capacity; i++) iota[i] = i;
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_ctrls(), z.data(), sizeof(InstCtrl) * capacity,
                           hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_iota(), iota.data(), sizeof(int32_t) * capacity,
                           hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->up_stream);
    if (e != hipSuccess) {
        err = std::string("init: ") + hipGetErrorString(e);
        ng_batch_destroy(b);
        return NG_EDEVICE;
    }
    *out = b;
    return NG_OK;
}

void fill_desc(InstDesc& d, const ng_gas* gas, const ng_grid* grid, const ng_numerics* num,
               int prec)
{
    memset(&d, 0, sizeof(d));
    d.nx = grid->nx;
    d.ny = grid->ndim == 2 ? grid->ny : 1;
    d.ncell = d.nx * d.ny;
    d.ndim = grid->ndim;
    d.riemann = num->riemann;
    d.scheme = num->scheme;
    d.any_bc = 0;
    for (int i = 0; i < 4; i++) {
        d.bc[i] = (i < 2 || grid->ndim == 2) ? grid->bc[i] : NG_BC_PERIODIC;
        if (d.bc[i] != NG_BC_PERIODIC) d.any_bc = 1;
    }
    d.h = grid->h;
    // an active wedge takes the boundary instantiation of the kernels
    d.wedge_tan = grid->wedge_tan > 0.0 ? grid->wedge_tan : 0.0;
    d.wedge_x0 = grid->wedge_x0;
    d.wedge_y0 = grid->wedge_y0;
    if (d.wedge_tan > 0.0) d.any_bc = 1;
    d.src_yc = grid->src_yc;
    d.src_hw = d.bc[0] == NG_BC_SOURCE && grid->src_hw > 0.0 ? grid->src_hw : 0.0;
    if (d.bc[0] == NG_BC_SOURCE) {
        // the forced wave's constants (the device evaluates the sine at each
        // accepted time)
        const double pi = 3.141592653589793;
        const double rho_b = gas->rho0;
        const double p_b = gas->R * gas->rho0 * gas->T0;
        // the ghosts lie before x = 0, outside any wedge (wedge_x0 >= 0): the
        // background there is the passive one when the grid has a wedge
        const double act = d.wedge_tan > 0.0 ? 0.0 : 1.0;
        const double ev_b = gas->rho0 * gas->Cv * gas->T0 + act * (gas->rho0 * gas->tau0 * gas->Q0);
        const double c = sqrt(gas->gamma * p_b / rho_b);
        d.src_amp = grid->src_amp;
        d.src_k = 2.0 * pi / grid->src_lambda;
        d.src_omega = c * d.src_k;
        d.src_rho = rho_b;
        d.src_p = p_b;
        d.src_ev = ev_b;
        d.src_uc = c / rho_b;
        d.src_c2 = c * c;
        d.src_er = ev_b / rho_b;
    }
    d.cfl = num->cfl;
    d.stiff_z = num->stiff_z;
    d.gamma = gas->gamma;
    d.gm1 = gas->gamma - 1.0;
    d.R = gas->R;
    d.Cv = gas->Cv;
    d.rho0 = gas->rho0;
    d.T0 = gas->T0;
    d.tau0 = gas->tau0;
    d.tau_rho = gas->tau_rho;
    d.tau_T = gas->tau_T;
    d.Q0 = gas->Q0;
    d.Q_rho = gas->Q_rho;
    d.Q_T = gas->Q_T;
    d.I0 = gas->I0;
    d.I_rho = gas->I_rho;
    d.I_T = gas->I_T;
    d.fx = gas->fx;
    d.fy = gas->fy;
    if (prec != NG_FP64) {
        // uniform reference at rest: rho0, p = R rho0 T0 and the vibrational
        // energy at which relaxation balances the pump in eq. (4)
        double rho_r = gas->rho0;
        double p_r = gas->R * gas->rho0 * gas->T0;
        double ev_r = gas->rho0 * gas->Cv * gas->T0 + gas->rho0 * gas->tau0 * gas->Q0;
        double E_r = p_r / d.gm1 + ev_r;
        d.uref[0] = rho_r;
        d.uref[3] = E_r;
        d.uref[4] = ev_r;
        d.p_r = p_r;
        d.e1_r = p_r / d.gm1;
        d.H_r = d.e1_r + p_r;
        d.D_r = gas->Cv / gas->R * p_r - ev_r;
    }
    // eq. (6) with T = p / (R rho): (rho/rho0)^x (T/T0)^y =
    // rho0^-x (R T0)^-y rho^(x - y) p^y; 1/tau takes the negated exponents
    const double RT0 = gas->R * gas->T0;
    const double xs[3] = {-gas->tau_rho, gas->Q_rho, gas->I_rho};
    const double ys[3] = {-gas->tau_T, gas->Q_T, gas->I_T};
    const double cs[3] = {1.0 / gas->tau0, gas->Q0, gas->I0};
    int codes[6];
    bool half = true;
    for (int i = 0; i < 3; i++) {
        d.cl_a[i] = xs[i] - ys[i];
        d.cl_b[i] = ys[i];
        d.cl_c[i] = cs[i] * pow(gas->rho0, -xs[i]) * pow(RT0, -ys[i]);
        for (int j = 0; j < 2; j++) {
            const double e2 = 2.0 * (j == 0 ? d.cl_a[i] : d.cl_b[i]);
            if (e2 != nearbyint(e2) || fabs(e2) > 4.0) half = false;
            else codes[2 * i + j] = (int)e2;
        }
    }
    d.cl_recipe = 0;
    for (int r = 1; half && r <= ng::kRecipes; r++) {
        bool same = true;
        for (int q = 0; q < 6; q++) same = same && codes[q] == ng::kRecipeCodes[r][q];
        if (same) d.cl_recipe = r;
    }
}

// Validate and upload a solve's conserved state into the slot's buffer 0, run
// the priming pass (first dt, totals, checks).  Synchronising.
int64_t small_limit_of(const ng_batch* b)
{
    return b->small_limit >= 0 ? b->small_limit
                               : (b->prec != NG_FP64 ? kSmallCells32 : kSmallCells64);
}

// Pinned staging of at least `bytes` (at most kStageBytes), both buffers idle.
int ensure_stage(ng_batch* b, size_t bytes)
{
    bytes = bytes < kStageBytes ? bytes : kStageBytes;
    if (b->stage_bytes >= bytes) return NG_OK;
    for (int k = 0; k < 2; k++) {
        CK(b, hipEventSynchronize(b->ev_stage[k]));
        if (b->stage[k]) CK(b, hipHostFree(b->stage[k]));
        b->stage[k] = nullptr;
    }
    b->stage_bytes = 0;
    for (int k = 0; k < 2; k++) CK(b, hipHostMalloc(&b->stage[k], bytes, 0));
    b->stage_bytes = bytes;
    return NG_OK;
}

// Convert cells [a, b) of a chunk starting at cell i0 of the caller's FP64
// state (primitive or conserved planes) to the stored form: FP64 conserved, or
// FP32 deviations from the reference.  Checks each cell (finite, rho > 0,
// p > 0); on failure returns the reason.
template <class R>
const char* convert_cells(const double* data, int64_t n, int nc, double gm1, const double* ref,
                          bool split, double e1_r, bool is_prim, int64_t i0, int64_t a, int64_t b,
                          R* st, int64_t m)
{
    double Wc[5], Uc[5];
    const int iE = nc == 5 ? 3 : 2, iV = nc - 1;
    for (int64_t i = a; i < b; i++) {
        for (int c = 0; c < nc; c++) (is_prim ? Wc : Uc)[c] = data[c * n + i0 + i];
        if (is_prim)
            prim_to_cons_cell(gm1, nc, Wc, Uc);
        else
            cons_to_prim_cell(gm1, nc, Uc, Wc);
        for (int c = 0; c < nc; c++) {
            if (!isfinite(Uc[c]) || !isfinite(Wc[c])) return "non-finite initial value";
            st[c * m + i] = (R)(Uc[c] - ref[c]);
        }
        // deviation storage keeps E - E_nu in the energy slot
        if (split) st[iE * m + i] = (R)((Uc[iE] - Uc[iV]) - e1_r);
        if (!(Wc[0] > 0.0) || !(Wc[nc == 5 ? 3 : 2] > 0.0))
            return "initial density and pressure must be positive";
    }
    return nullptr;
}

// Convert the initial state chunk by chunk into the pinned staging (large
// chunks split over host threads) and copy each chunk to buffer 0 of the solve
// on the upload stream.
template <class R>
int upload_state(ng_batch* b, const Slot& s, const double* data, bool is_prim)
{
    const int nc = ncomp(s.dim);
    const int64_t n = s.d.ncell;
    const double gm1 = s.d.gm1;
    const double ref5[5] = {s.d.uref[0], 0.0, 0.0, s.d.uref[3], s.d.uref[4]};
    const double ref4[4] = {s.d.uref[0], 0.0, s.d.uref[3], s.d.uref[4]};
    const double* ref = nc == 5 ? ref5 : ref4;
    const bool split = b->prec != NG_FP64;
    int rc = ensure_stage(b, sizeof(R) * nc * (size_t)n);
    if (rc) return rc;
    const int64_t per = (int64_t)(b->stage_bytes / (sizeof(R) * nc));
    char* dst = (char*)s.d.buf[0];
    const int hw = (int)std::thread::hardware_concurrency();
    const int max_threads = hw < 1 ? 1 : (hw > kHostThreads ? kHostThreads : hw);
    int k = 0;
    for (int64_t i0 = 0; i0 < n; i0 += per, k ^= 1) {
        const int64_t m = n - i0 < per ? n - i0 : per;
        CK(b, hipEventSynchronize(b->ev_stage[k]));
        R* st = (R*)b->stage[k];
        int nt = (int)(m / kCellsPerThread);
        nt = nt < 1 ? 1 : (nt > max_threads ? max_threads : nt);
        std::vector<const char*> why(nt, nullptr);
        if (nt == 1) {
            why[0] = convert_cells<R>(data, n, nc, gm1, ref, split, s.d.e1_r, is_prim, i0, 0, m, st,
                                     m);
        } else {
            std::vector<std::thread> th;
            for (int t = 0; t < nt; t++)
                th.emplace_back([&, t] {
                    why[t] = convert_cells<R>(data, n, nc, gm1, ref, split, s.d.e1_r, is_prim,
                                              i0, m * t / nt, m * (t + 1) / nt, st, m);
                });
            for (auto& x : th) x.join();
        }
        for (const char* w : why)
            if (w) {
                b->err = w;
                return NG_EINVAL;
            }
        for (int c = 0; c < nc; c++)
            CK(b, hipMemcpyAsync(dst + sizeof(R) * (c * n + i0), st + c * m, sizeof(R) * m,
                                 hipMemcpyHostToDevice, b->up_stream));
        CK(b, hipEventRecord(b->ev_stage[k], b->up_stream));
    }
    return NG_OK;
}

// Admit a solve.  The host converts and checks the initial state while the
// steps already enqueued run; the upload goes on the upload stream, and the
// priming pass of this solve (its totals, signal speed and first dt) is
// enqueued on the batch stream behind it.  The solve joins the per-step
// launches at the next run (the tables are rebuilt then).  Nothing here waits
// for the batch stream.
int add_solve(ng_batch* b, const ng_gas* gas, const ng_grid* grid, const ng_numerics* num,
              const double* data, bool is_prim, double t0, double t_end, int64_t max_steps,
              int32_t* slot_out)
{
    std::string err;
    int rc = validate(gas, grid, num, err);
    if (rc) {
        b->err = err;
        return rc;
    }
    if (num->precision != b->prec) {
        b->err = "precision differs from the batch";
        return NG_EINVAL;
    }
    if (!data || !isfinite(t0) || !(t_end > t0) || max_steps < 0) {
        b->err = "invalid state pointer, t0, t_end or max_steps";
        return NG_EINVAL;
    }
    int slot = -1;
    for (int i = 0; i < b->capacity; i++)
        if (!b->slots[i].live) {
            slot = i;
            break;
        }
    if (slot < 0) {
        b->err = "no free slot";
        return NG_EFULL;
    }
    const size_t sb = solve_bytes(grid, b->prec);
    size_t off = 0;
    if (!arena_alloc(b, sb, &off)) {
        b->err = "no room in the device arena";
        return NG_EFULL;
    }
    Slot& s = b->slots[slot];
    s = Slot();
    s.dim = grid->ndim;
    s.off = off;
    s.bytes = sb;
    s.partial_cap = partial_cap_of(grid);
    fill_desc(s.d, gas, grid, num, b->prec);
    const size_t pb = state_plane_bytes(grid, b->prec);
    s.d.buf[0] = (uint64_t)(b->arena + off);
    s.d.buf[1] = (uint64_t)(b->arena + off + pb);
    s.d.partials = (uint64_t)(b->arena + off + 2 * pb);
    s.small = s.d.ncell <= small_limit_of(b);
    shape_solve(b, s);
    auto fail = [&](int code) {
        // copies of this solve may still be queued: let them land before the
        // arena block can be handed out again
        (void)hipStreamSynchronize(b->up_stream);
        arena_free(b, off, sb);
        s = Slot();
        return code;
    };
    if (s.d.nblocks > s.partial_cap) {
        b->err = "launch shape needs more reduction records than reserved";
        return fail(NG_EINVAL);
    }
    // the previous admission's copies have left the per-slot staging
    hipError_t e = hipEventSynchronize(b->ev_ready);
    if (e != hipSuccess) return fail(dev_err(b, e, "hipEventSynchronize"));
    rc = b->prec == NG_FP32 ? upload_state<float>(b, s, data, is_prim)
                            : upload_state<double>(b, s, data, is_prim);
    if (rc) return fail(rc);
    InstCtrl& c = b->h_ctrl_up[slot];
    memset(&c, 0, sizeof(c));
    c.t = t0;
    c.t_end = t_end;
    c.max_steps = max_steps;
    b->h_desc_up[slot] = s.d;
    e = hipMemcpyAsync(b->d_descs() + slot, &b->h_desc_up[slot], sizeof(InstDesc),
                       hipMemcpyHostToDevice, b->up_stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_ctrls() + slot, &c, sizeof(InstCtrl), hipMemcpyHostToDevice,
                           b->up_stream);
    if (e == hipSuccess) e = hipEventRecord(b->ev_ready, b->up_stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(b->stream, b->ev_ready, 0);
    if (e != hipSuccess) return fail(dev_err(b, e, "upload"));
    // priming pass over this solve only: its own workgroups, listed by index
    e = launch_prime(s.dim, kind_of(b->prec), b->d_descs(), b->d_ctrls(), nullptr, slot,
                     s.d.nblocks, s.d.waves_per_block, b->stream);
    if (e == hipSuccess)
        e = launch_finalize(b->d_descs(), b->d_ctrls(), b->d_iota() + slot, 1, 1, b->stream);
    if (e != hipSuccess) {
        (void)hipStreamSynchronize(b->stream);
        return fail(dev_err(b, e, "prime"));
    }
    s.live = true;
    b->dirty = true;
    *slot_out = slot;
    return NG_OK;
}

int read_conserved(ng_batch* b, int slot, double* out, bool prim)
{
    if (slot < 0 || slot >= b->capacity || !b->slots[slot].live || !out) {
        b->err = "invalid slot or output";
        return NG_EINVAL;
    }
    int rc = read_ctrls(b);
    if (rc) return rc;
    Slot& s = b->slots[slot];
    const int nc = ncomp(s.dim);
    const int64_t n = s.d.ncell;
    const int cur = b->h_ctrls[slot].cur;
    std::vector<double> U((size_t)nc * n);
    if (b->prec != NG_FP32) {
        // FP64 state (deviations from the reference for the mixed path)
        CK(b, hipMemcpy(U.data(), (void*)s.d.buf[cur], sizeof(double) * U.size(),
                        hipMemcpyDeviceToHost));
        if (b->prec == NG_MIXED) {
            const double ref5[5] = {s.d.uref[0], 0.0, 0.0, s.d.e1_r, s.d.uref[4]};
            const double ref4[4] = {s.d.uref[0], 0.0, s.d.e1_r, s.d.uref[4]};
            const double* ref = nc == 5 ? ref5 : ref4;
            for (int c = 0; c < nc; c++)
                for (int64_t i = 0; i < n; i++) U[c * n + i] += ref[c];
        }
    } else {
        std::vector<float> D((size_t)nc * n);
        CK(b, hipMemcpy(D.data(), (void*)s.d.buf[cur], sizeof(float) * D.size(),
                        hipMemcpyDeviceToHost));
        const double ref5[5] = {s.d.uref[0], 0.0, 0.0, s.d.e1_r, s.d.uref[4]};
        const double ref4[4] = {s.d.uref[0], 0.0, s.d.e1_r, s.d.uref[4]};
        const double* ref = nc == 5 ? ref5 : ref4;
        for (int c = 0; c < nc; c++)
            for (int64_t i = 0; i < n; i++) U[c * n + i] = ref[c] + (double)D[c * n + i];
    }
    if (b->prec != NG_FP64) {
        // the energy slot held E - E_nu
        const int iE = nc == 5 ? 3 : 2, iV = nc - 1;
        for (int64_t i = 0; i < n; i++) U[iE * n + i] += U[iV * n + i];
    }
    if (!prim) {
        memcpy(out, U.data(), sizeof(double) * U.size());
        return NG_OK;
    }
    double Uc[5], Wc[5];
    for (int64_t i = 0; i < n; i++) {
        for (int c = 0; c < nc; c++) Uc[c] = U[c * n + i];
        cons_to_prim_cell(s.d.gm1, nc, Uc, Wc);
        for (int c = 0; c < nc; c++) out[c * n + i] = Wc[c];
    }
    return NG_OK;
}

int diag_of(ng_batch* b, int slot, ng_diag* out)
{
    if (slot < 0 || slot >= b->capacity || !b->slots[slot].live || !out) {
        b->err = "invalid slot or output";
        return NG_EINVAL;
    }
    int rc = read_ctrls(b);
    if (rc) return rc;
    const InstCtrl& c = b->h_ctrls[slot];
    const Slot& s = b->slots[slot];
    double hd = s.dim == 2 ? s.d.h * s.d.h : s.d.h;
    memset(out, 0, sizeof(*out));
    out->t = c.t;
    out->dt_last = c.dt_last;
    double dt = c.dt_cfl;
    if (c.t + dt > c.t_end) dt = c.t_end - c.t;
    out->dt_next = dt;
    out->steps = c.steps;
    for (int q = 0; q < 5; q++) out->total[q] = c.total[q] * hd;
    out->src_budget[0] = c.budget[0] * hd;
    out->src_budget[1] = c.budget[1] * hd;
    out->rho_min = c.rho_min;
    out->p_min = c.p_min;
    out->smax = c.smax;
    out->status = c.status;
    out->flags = c.flags;
    if (c.status == 0 && (!(c.t < c.t_end) || c.steps >= c.max_steps)) out->flags |= NG_FLAG_DONE;
    return NG_OK;
}

}  // namespace

// ===================================================================== C ABI

extern "C" {

const char* ng_strerror(int code)
{
    switch (code) {
    case NG_OK: return "ok";
    case NG_EINVAL: return "invalid argument";
    case NG_ENOMEM: return "device buffer too small";
    case NG_EPHYS: return "non-physical state (rho <= 0, p <= 0 or non-finite)";
    case NG_EDEVICE: return "HIP runtime error";
    case NG_EFULL: return "batch full";
    case NG_ESTALL: return "cooperative launch stalled (grid-barrier wait ran out of polls)";
    default: return "unknown error";
    }
}

int ng_state_bytes(const ng_grid* grid, const ng_numerics* num, size_t* bytes)
{
    if (!grid || !num || !bytes) return NG_EINVAL;
    if (grid->ndim != 1 && grid->ndim != 2) return NG_EINVAL;
    if (grid->nx < 4 || (grid->ndim == 2 && grid->ny < 4) || (grid->ndim == 1 && grid->ny != 1))
        return NG_EINVAL;
    if (!prec_ok(num->precision)) return NG_EINVAL;
    size_t tc = (size_t)partial_cap_of(grid);
    Layout L = header_layout(1, grid->ndim == 1 ? tc : 0, grid->ndim == 2 ? tc : 0);
    *bytes = L.heap + solve_bytes(grid, num->precision);
    return NG_OK;
}

static int solver_new(const ng_gas* gas, const ng_grid* grid, const ng_numerics* num,
                      const double* data, bool is_prim, double t0, void* dev_buf,
                      size_t dev_bytes, void* hip_stream, ng_solver** out)
{
    if (!out) return NG_EINVAL;
    *out = nullptr;
    std::string err;
    int rc = validate(gas, grid, num, err);
    if (rc) return rc;
    size_t need = 0;
    rc = ng_state_bytes(grid, num, &need);
    if (rc) return rc;
    if (dev_bytes < need) return NG_ENOMEM;
    size_t tc = (size_t)partial_cap_of(grid);
    ng_batch* b = nullptr;
    rc = batch_new(1, num->precision, dev_buf, need, hip_stream, grid->ndim == 1 ? tc : 0,
                   grid->ndim == 2 ? tc : 0, &b, err);
    if (rc) return rc;
    int32_t slot = 0;
    rc = add_solve(b, gas, grid, num, data, is_prim, t0, INFINITY, INT64_MAX, &slot);
    if (!rc) rc = read_ctrls(b);
    if (!rc && b->h_ctrls[slot].status != 0) rc = NG_EPHYS;
    if (rc) {
        ng_batch_destroy(b);
        return rc;
    }
    ng_solver* s = new ng_solver();
    s->b = b;
    s->slot = slot;
    *out = s;
    return NG_OK;
}

int ng_init_state(const ng_gas* gas, const ng_grid* grid, const ng_numerics* num,
                  const double* prim, double t0, void* dev_buf, size_t dev_bytes,
                  void* hip_stream, ng_solver** out)
{
    return solver_new(gas, grid, num, prim, true, t0, dev_buf, dev_bytes, hip_stream, out);
}

int ng_init_conserved(const ng_gas* gas, const ng_grid* grid, const ng_numerics* num,
                      const double* cons, double t0, void* dev_buf, size_t dev_bytes,
                      void* hip_stream, ng_solver** out)
{
    return solver_new(gas, grid, num, cons, false, t0, dev_buf, dev_bytes, hip_stream, out);
}

static int solver_rc(ng_solver* s, int rc)
{
    if (rc && s) s->err = s->b->err;
    return rc;
}

int ng_step(ng_solver* s, int64_t nsteps)
{
    if (!s || nsteps < 0) return NG_EINVAL;
    if (nsteps == 0) return NG_OK;
    std::vector<int32_t> sl{s->slot};
    int rc = set_limits(s->b, sl, INFINITY, -1);
    if (!rc) rc = enqueue_steps(s->b, nsteps);
    return solver_rc(s, rc);
}

int ng_run_to_time(ng_solver* s, double t_end, int64_t max_steps, int64_t* steps_taken)
{
    if (!s || !isfinite(t_end) || max_steps < 0) return NG_EINVAL;
    ng_batch* b = s->b;
    int rc = read_ctrls(b);
    if (rc) return solver_rc(s, rc);
    const int64_t steps0 = b->h_ctrls[s->slot].steps;
    std::vector<int32_t> sl{s->slot};
    rc = set_limits(b, sl, t_end, max_steps);
    if (rc) return solver_rc(s, rc);
    for (;;) {
        rc = read_ctrls(b);
        if (rc) return solver_rc(s, rc);
        const InstCtrl& c = b->h_ctrls[s->slot];
        if (c.status != 0) {
            if (steps_taken) *steps_taken = c.steps - steps0;
            if (c.status == kStatusStall) {
                s->err = "cooperative launch: a grid-barrier wait ran out of polls";
                return NG_ESTALL;
            }
            s->err = "step rejected: non-physical state";
            return NG_EPHYS;
        }
        int64_t left = max_steps - (c.steps - steps0);
        if (!(c.t < t_end) || left <= 0) {
            if (steps_taken) *steps_taken = c.steps - steps0;
            return NG_OK;
        }
        // estimate of the steps still needed; the device stops by itself
        double est = c.dt_cfl > 0.0 ? (t_end - c.t) / c.dt_cfl : (double)left;
        int64_t chunk = (int64_t)std::min<double>((double)left, ceil(est * 1.02) + 1.0);
        if (chunk < 1) chunk = 1;
        rc = enqueue_steps(b, chunk);
        if (rc) return solver_rc(s, rc);
    }
}

int ng_diagnostics(ng_solver* s, ng_diag* out)
{
    if (!s) return NG_EINVAL;
    return solver_rc(s, diag_of(s->b, s->slot, out));
}

int ng_get_state(ng_solver* s, double* prim_out)
{
    if (!s) return NG_EINVAL;
    return solver_rc(s, read_conserved(s->b, s->slot, prim_out, true));
}

int ng_get_conserved(ng_solver* s, double* cons_out)
{
    if (!s) return NG_EINVAL;
    return solver_rc(s, read_conserved(s->b, s->slot, cons_out, false));
}

int ng_set_launch(ng_solver* s, int32_t rows_per_item, int32_t waves_per_block)
{
    if (!s) return NG_EINVAL;
    return ng_batch_set_launch(s->b, s->b->slots[s->slot].dim, rows_per_item, waves_per_block);
}

int ng_batch_set_fused_accept(ng_batch* b, int32_t on)
{
    if (!b) return NG_EINVAL;
    b->fused = on != 0;
    b->dirty = true;
    return rebuild(b);
}

int ng_set_fused_accept(ng_solver* s, int32_t on)
{
    if (!s) return NG_EINVAL;
    return ng_batch_set_fused_accept(s->b, on);
}

int ng_set_small_limit(ng_solver* s, int64_t max_cells)
{
    if (!s) return NG_EINVAL;
    return solver_rc(s, ng_batch_set_small_limit(s->b, max_cells));
}

int ng_set_coop(ng_solver* s, int64_t max_cells, int32_t spin_limit)
{
    if (!s) return NG_EINVAL;
    return solver_rc(s, ng_batch_set_coop(s->b, max_cells, spin_limit));
}

int ng_set_graph_steps(ng_solver* s, int32_t steps)
{
    if (!s || steps < 1 || steps > 4096) return NG_EINVAL;
    s->b->graph_steps = steps;
    drop_graph(s->b);
    return NG_OK;
}

int ng_enable_timing(ng_solver* s, int32_t nsteps, int32_t every)
{
    if (!s || nsteps < 0 || every < 1) return NG_EINVAL;
    s->b->timing = nsteps != 0;
    s->b->timing_every = every;
    // 2 around a persistent launch, 4 per timed step and dimension
    size_t need = nsteps ? 2 + ((size_t)nsteps + every - 1) / every * 4 * 2 : 0;
    if (need && !get_event(s->b, need - 1)) return solver_rc(s, dev_err(s->b, hipErrorOutOfMemory, "hipEventCreate"));
    return NG_OK;
}

int ng_kernel_time(ng_solver* s, double* step_ms, double* finalize_ms, int64_t* launches)
{
    if (!s) return NG_EINVAL;
    if (step_ms) *step_ms = s->b->t_step_ms;
    if (finalize_ms) *finalize_ms = s->b->t_fin_ms;
    if (launches) *launches = s->b->t_launches;
    return NG_OK;
}

// --------------------------------------------- one step without allocation

// The entry point for callers that cannot allocate: one FP64 step from U_in to
// U_out with the descriptor, control block, workgroup table and reduction
// records in the library's static scratch (ng_kernels.hip).  The launch shape
// is the automatic one of a lone solve, so the state equals ng_step's.
static thread_local std::string g_static_err;

int ng_step_static(const ng_gas* gas, const ng_grid* grid, const ng_numerics* num,
                   const void* U_in, void* U_out, double t, double t_end, void* hip_stream,
                   ng_diag* out)
{
    std::string err;
    int rc = validate(gas, grid, num, err);
    if (rc) {
        g_static_err = err;
        return rc;
    }
    if (num->precision != NG_FP64) {
        g_static_err = "ng_step_static: the state must be FP64 (NG_FP64)";
        return NG_EINVAL;
    }
    if (!U_in || !U_out || U_in == (const void*)U_out) {
        g_static_err = "ng_step_static: U_in and U_out must be distinct device buffers";
        return NG_EINVAL;
    }
    InstDesc d;
    fill_desc(d, gas, grid, num, NG_FP64);
    const int dim = grid->ndim;
    d.rows_per_item = auto_rows(dim, {{d.nx, d.ny}});
    d.nstrips = (int32_t)cdiv(d.nx, dim == 2 ? kInterior : seg_cells(d.scheme));
    d.nchunks = (int32_t)(dim == 2 ? cdiv(d.ny, d.rows_per_item) : cdiv(d.nstrips, d.rows_per_item));
    d.nitems = dim == 2 ? (int64_t)d.nstrips * d.nchunks : (int64_t)d.nchunks;
    d.waves_per_block = dim == 2 ? kDefaultWaves2D : (d.nitems < kAutoItems1DWaves ? 2 : 4);
    d.nblocks = cdiv(d.nitems, d.waves_per_block);
    d.fused = d.nblocks <= kFusedMaxBlocks ? 1 : 0;
    // scratch layout: descriptor, control block, finalize index list,
    // workgroup table, per-workgroup records
    const size_t o_ctrl = align_up(sizeof(InstDesc));
    const size_t o_insts = o_ctrl + align_up(sizeof(InstCtrl));
    const size_t o_blocks = o_insts + kAlign;
    const size_t o_parts = o_blocks + align_up(sizeof(BlockRef) * (size_t)d.nblocks);
    const size_t need = o_parts + sizeof(Partial) * (size_t)d.nblocks;
    if (need > kStaticScratchBytes) {
        g_static_err = "ng_step_static: the grid needs " + std::to_string(need) +
                       " bytes of scratch (" + std::to_string(d.nblocks) +
                       " workgroups), the static scratch holds " +
                       std::to_string(kStaticScratchBytes);
        return NG_ENOMEM;
    }
    void* base = nullptr;
    hipError_t e = static_scratch(&base);
    if (e != hipSuccess) {
        g_static_err = std::string("hipGetSymbolAddress: ") + hipGetErrorString(e);
        return NG_EDEVICE;
    }
    char* sc = (char*)base;
    InstDesc* descs = (InstDesc*)sc;
    InstCtrl* ctrls = (InstCtrl*)(sc + o_ctrl);
    int32_t* insts = (int32_t*)(sc + o_insts);
    BlockRef* blocks = (BlockRef*)(sc + o_blocks);
    d.buf[0] = (uint64_t)(uintptr_t)U_in;
    d.buf[1] = (uint64_t)(uintptr_t)U_out;
    d.partials = (uint64_t)(uintptr_t)(sc + o_parts);
    InstCtrl c;
    memset(&c, 0, sizeof(c));
    c.t = t;
    c.t_end = t_end > t ? t_end : INFINITY;
    c.max_steps = 1;
    const int variant = d.scheme == kSchemeCsph ? kVariantCsph
                                                : ((d.riemann == NG_HLLC && !d.any_bc) ? 1 : 0);
    hipStream_t st = (hipStream_t)hip_stream;
    e = launch_static_setup(d, c, descs, ctrls, insts, blocks, d.nblocks, st);
    if (e == hipSuccess)
        e = launch_prime(dim, kind_of(NG_FP64), descs, ctrls, nullptr, 0, d.nblocks,
                         d.waves_per_block, st);
    if (e == hipSuccess) e = launch_finalize(descs, ctrls, insts, 1, 1, st);
    if (e == hipSuccess)
        e = launch_step(dim, kind_of(NG_FP64), variant, descs, ctrls, blocks, d.nblocks,
                        d.waves_per_block, 1, d.fused, st);
    if (e == hipSuccess && !d.fused) e = launch_finalize(descs, ctrls, insts, 1, 0, st);
    if (e != hipSuccess) {
        g_static_err = std::string("kernel launch: ") + hipGetErrorString(e);
        return NG_EDEVICE;
    }
    if (!out) return NG_OK;
    InstCtrl h;
    e = hipMemcpyAsync(&h, ctrls, sizeof(InstCtrl), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        g_static_err = std::string("read-back: ") + hipGetErrorString(e);
        return NG_EDEVICE;
    }
    const double hd = dim == 2 ? d.h * d.h : d.h;
    memset(out, 0, sizeof(*out));
    out->t = h.t;
    out->dt_last = h.dt_last;
    double dt = h.dt_cfl;
    if (h.t + dt > h.t_end) dt = h.t_end - h.t;
    out->dt_next = dt;
    out->steps = h.steps;
    for (int q = 0; q < 5; q++) out->total[q] = h.total[q] * hd;
    out->src_budget[0] = h.budget[0] * hd;
    out->src_budget[1] = h.budget[1] * hd;
    out->rho_min = h.rho_min;
    out->p_min = h.p_min;
    out->smax = h.smax;
    out->status = h.status;
    out->flags = h.flags;
    if (h.status != 0) {
        g_static_err = "ng_step_static: the step produced rho <= 0, p <= 0 or a non-finite value";
        return NG_EPHYS;
    }
    return NG_OK;
}

const char* ng_static_last_error(void) { return g_static_err.c_str(); }

const char* ng_last_error(const ng_solver* s)
{
    if (!s) return "null solver";
    return s->err.empty() ? s->b->err.c_str() : s->err.c_str();
}

void ng_destroy(ng_solver* s)
{
    if (!s) return;
    ng_batch_destroy(s->b);
    delete s;
}

// ------------------------------------------------------------------- batch

int ng_batch_create(int32_t capacity, int32_t precision, void* dev_buf, size_t dev_bytes,
                    void* hip_stream, ng_batch** out)
{
    if (!out) return NG_EINVAL;
    *out = nullptr;
    // workgroup tables: at most one entry per 60 cells of a 1D solve (the
    // densest decomposition); bound them by the arena size
    size_t per = 60 * 2 * 4 * (precision == NG_FP32 ? 4 : 8);
    size_t tcap = dev_bytes / per + 64 * (size_t)capacity;
    std::string err;
    return batch_new(capacity, precision, dev_buf, dev_bytes, hip_stream, tcap, tcap / 4 + 64 * capacity,
                     out, err);
}

int ng_batch_solve_bytes(const ng_grid* grid, int32_t precision, size_t* bytes)
{
    if (!grid || !bytes || (grid->ndim != 1 && grid->ndim != 2)) return NG_EINVAL;
    if (!prec_ok(precision)) return NG_EINVAL;
    *bytes = solve_bytes(grid, precision);
    return NG_OK;
}

int ng_batch_fits(const ng_batch* b, const ng_grid* grid, int32_t* fits)
{
    if (!b || !grid || !fits || (grid->ndim != 1 && grid->ndim != 2)) return NG_EINVAL;
    if (grid->nx < 1 || (grid->ndim == 2 && grid->ny < 1)) return NG_EINVAL;
    *fits = has_room(b, solve_bytes(grid, b->prec)) ? 1 : 0;
    return NG_OK;
}

int ng_batch_add(ng_batch* b, const ng_gas* gas, const ng_grid* grid, const ng_numerics* num,
                 const double* prim, double t0, double t_end, int64_t max_steps, int32_t* slot)
{
    if (!b || !slot) return NG_EINVAL;
    if (!isfinite(t_end)) {
        b->err = "t_end must be finite";
        return NG_EINVAL;
    }
    return add_solve(b, gas, grid, num, prim, true, t0, t_end, max_steps, slot);
}

int ng_batch_run(ng_batch* b, int64_t nsteps)
{
    if (!b || nsteps < 0) return NG_EINVAL;
    return enqueue_steps(b, nsteps);
}

int ng_batch_poll(ng_batch* b, int32_t* done_slots, int32_t cap, int32_t* ndone)
{
    if (!b || !ndone || (cap > 0 && !done_slots)) return NG_EINVAL;
    int rc = read_ctrls(b);
    if (rc) return rc;
    int32_t n = 0;
    for (int i = 0; i < b->capacity && n < cap; i++) {
        Slot& s = b->slots[i];
        if (!s.live || s.reported) continue;
        const InstCtrl& c = b->h_ctrls[i];
        bool fin = c.status != 0 || !(c.t < c.t_end) || c.steps >= c.max_steps;
        if (fin) {
            s.reported = true;
            done_slots[n++] = i;
        }
    }
    *ndone = n;
    return NG_OK;
}

int ng_batch_active(ng_batch* b, int32_t* nactive)
{
    if (!b || !nactive) return NG_EINVAL;
    int rc = read_ctrls(b);
    if (rc) return rc;
    int32_t n = 0;
    for (int i = 0; i < b->capacity; i++) {
        if (!b->slots[i].live) continue;
        const InstCtrl& c = b->h_ctrls[i];
        if (c.status == 0 && c.t < c.t_end && c.steps < c.max_steps) n++;
    }
    *nactive = n;
    return NG_OK;
}

int ng_batch_diagnostics(ng_batch* b, int32_t slot, ng_diag* out)
{
    if (!b) return NG_EINVAL;
    return diag_of(b, slot, out);
}

int ng_batch_get_state(ng_batch* b, int32_t slot, double* prim_out)
{
    if (!b) return NG_EINVAL;
    return read_conserved(b, slot, prim_out, true);
}

int ng_batch_get_conserved(ng_batch* b, int32_t slot, double* cons_out)
{
    if (!b) return NG_EINVAL;
    return read_conserved(b, slot, cons_out, false);
}

int ng_batch_remove(ng_batch* b, int32_t slot)
{
    if (!b || slot < 0 || slot >= b->capacity || !b->slots[slot].live) return NG_EINVAL;
    // nothing of this solve may still be in flight
    hipError_t e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return dev_err(b, e, "hipStreamSynchronize");
    Slot& s = b->slots[slot];
    arena_free(b, s.off, s.bytes);
    s = Slot();
    InstCtrl c;
    memset(&c, 0, sizeof(c));
    c.status = -1;
    e = hipMemcpyAsync(b->d_ctrls() + slot, &c, sizeof(c), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return dev_err(b, e, "remove");
    b->dirty = true;
    return NG_OK;
}

int ng_batch_set_launch(ng_batch* b, int32_t dim, int32_t rows_per_item, int32_t waves_per_block)
{
    if (!b || (dim != 1 && dim != 2)) return NG_EINVAL;
    if (rows_per_item < kAutoRows || waves_per_block < kAutoRows || waves_per_block > 4 ||
        (waves_per_block > 0 && (waves_per_block & (waves_per_block - 1))))
        return NG_EINVAL;
    if (dim == 2 && rows_per_item > 0 && rows_per_item < kMinRows2D) return NG_EINVAL;
    int old_r = b->rows[dim], old_w = b->waves[dim];
    if (rows_per_item) b->rows[dim] = rows_per_item;
    if (waves_per_block) b->waves[dim] = waves_per_block;
    b->dirty = true;
    int rc = rebuild(b);
    if (rc) {
        b->rows[dim] = old_r;
        b->waves[dim] = old_w;
        b->dirty = true;
        (void)rebuild(b);
        return rc;
    }
    return NG_OK;
}

int ng_batch_set_small_limit(ng_batch* b, int64_t max_cells)
{
    if (!b || max_cells < -1) return NG_EINVAL;
    b->small_limit = max_cells;
    b->dirty = true;
    return rebuild(b);
}

int ng_batch_set_coop(ng_batch* b, int64_t max_cells, int32_t spin_limit)
{
    if (!b || max_cells < -1 || spin_limit < -1) return NG_EINVAL;
    b->coop_limit = max_cells;
    b->coop_spin = spin_limit < 0 ? kCoopSpin : spin_limit;
    b->dirty = true;
    return rebuild(b);
}

const char* ng_batch_last_error(const ng_batch* b) { return b ? b->err.c_str() : "null batch"; }

void ng_batch_destroy(ng_batch* b)
{
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    drop_graph(b);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    for (auto e : b->ev_pool) (void)hipEventDestroy(e);
    if (b->up_stream) (void)hipStreamSynchronize(b->up_stream);
    if (b->h_ctrls) (void)hipHostFree(b->h_ctrls);
    if (b->h_desc_up) (void)hipHostFree(b->h_desc_up);
    if (b->h_ctrl_up) (void)hipHostFree(b->h_ctrl_up);
    for (int k = 0; k < 2; k++) {
        if (b->stage[k]) (void)hipHostFree(b->stage[k]);
        if (b->ev_stage[k]) (void)hipEventDestroy(b->ev_stage[k]);
    }
    if (b->ev_ready) (void)hipEventDestroy(b->ev_ready);
    if (b->up_stream) (void)hipStreamDestroy(b->up_stream);
    delete b;
}

}  // extern "C"
