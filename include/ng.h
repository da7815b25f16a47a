/*
 * ng.h -- C ABI of the MI355X (gfx950) library for the Eulerian MUSCL step of a
 * vibrationally excited gas.
 *
 * Method: S. S. Khrapov and A. V. Khoperskov, "Dynamics of unstable sound
 * waves in a non-equilibrium medium at the nonlinear stage", J. Phys.: Conf.
 * Ser. 973 (2018) 012007, arXiv:1805.03442.  The model is eqs. (1)-(5)
 * (continuity, momentum, total energy, vibrational energy) with the closures
 * (6) and the ideal-gas EOS (7); the step is the MUSCL predictor-corrector of
 * eq. (15) with the limited linear face states of eq. (14) (xi = 0), the HLL
 * flux of eq. (13) or the HLLC flux, and the time step of eq. (16).  1D
 * solves can take the paper's other step instead, CSPH-TVD (section 2.3,
 * eqs. (9)-(14)): a Lagrangian SPH predictor-corrector followed by an
 * Eulerian HLL remap of the displaced particles (ng_numerics.scheme).
 *
 * Conventions for every call:
 *   - return NG_OK (0) on success or a negative NG_E* code; the text of the
 *     last failure of an object is available from ng_last_error /
 *     ng_batch_last_error (NULL objects: ng_strerror of the code);
 *   - host pointers are plain C arrays owned by the caller; they are read or
 *     written only during the call;
 *   - device memory (dev_buf) and the HIP stream (hip_stream, a hipStream_t,
 *     NULL = the default stream) are owned by the caller and must outlive the
 *     object; the library never allocates or frees device memory other than
 *     a few bytes of pinned host memory for status read-back;
 *   - work is enqueued on the caller's stream; calls documented as
 *     "synchronising" wait for the stream; errors raised inside kernels
 *     (non-positive density or pressure, non-finite values) are reported by the
 *     next synchronising call as NG_EPHYS, and the object keeps the last state
 *     that passed the check;
 *   - objects are not thread-safe: one thread per object.
 *
 * Layout of the host state arrays (initial data and read-out): FP64, one plane
 * per component, cell (j, k) at index k * nx + j, centred at ((j + 1/2) h,
 * (k + 1/2) h).  Primitive arrays are (rho, u, [v], p, E_nu); conserved arrays
 * are (rho, rho u, [rho v], E, E_nu); 1D problems have no v plane (4 planes),
 * 2D problems have 5.
 */
#ifndef NG_H
#define NG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------- error codes */
#define NG_OK 0
#define NG_EINVAL (-1)  /* invalid argument or parameter                      */
#define NG_ENOMEM (-2)  /* device buffer smaller than required                 */
#define NG_EPHYS (-3)   /* a step produced rho <= 0, p <= 0 or a non-finite value */
#define NG_EDEVICE (-4) /* a HIP runtime call failed                           */
#define NG_EFULL (-5)   /* batch: no free slot or no room in the arena         */
#define NG_ESTALL (-6)  /* a cooperative launch's grid-barrier wait ran out of
                           polls (see ng_set_coop); the solve keeps its last
                           accepted step and stops, like NG_EPHYS              */

/* ------------------------------------------------------- enumerated options */
#define NG_BC_PERIODIC 0 /* wrap-around ghost cells                             */
#define NG_BC_WALL 1     /* reflecting wall: mirrored ghosts, normal momentum
                            negated (the solid walls of section 2.4)          */
#define NG_BC_OUTFLOW 2  /* free outflow: ghosts copy the edge cell           */
#define NG_BC_SOURCE 3   /* x-low end only: forced oscillations from a source
                            (the 1D runs of section 3): the ghosts carry the
                            plane sound wave of ng_grid.src_amp/src_lambda   */
#define NG_HLLC 0        /* three-wave HLLC flux (contact resolved)            */
#define NG_HLL 1         /* two-wave HLL flux, eq. (13)                         */
#define NG_MINMOD 0      /* minmod-limited slopes in eq. (14)                   */
#define NG_FP64 0        /* state, flux and sources in FP64                     */
#define NG_FP32 1        /* FP32 deviations from a uniform reference state,
                            FP64 totals and FP64 stiff relaxation factor      */
#define NG_MIXED 2       /* as NG_FP32, but the deviations are stored in FP64
                            and each step's FP32 increment is added in FP64   */
#define NG_MUSCL 0       /* the Eulerian MUSCL step of eq. (15)                 */
#define NG_CSPH_TVD 1    /* the CSPH-TVD step of section 2.3 (1D, NG_FP64,
                            NG_HLL): particles at the cell
                            centres move by the predictor (10) and corrector
                            (11) under eq. (12) -- SPH pressure force and work
                            over the two neighbours with the cubic-spline
                            kernel W of smoothing length h and particle volume
                            h, phi = sqrt(2 p); body force, pump, sink and
                            relaxation as in eqs. (2)-(4) -- and are remapped
                            by eq. (9) with the HLL flux (13) of u U between
                            the displaced face values of eq. (14), U^{n+1/2} =
                            (U^n + U~)/2, Theta the minmod slopes of U^n per
                            unit length.  Sources are explicit (stiff_z is not
                            used: the relaxation of eq. (4) is stable while
                            dt/tau stays below about 2, else the step fails
                            with NG_EPHYS); the time step is that of eq. (16).
                            Every
                            path of a 1D solve takes it (per-step, persistent,
                            cooperative, batches, ng_step_static)             */

/* status flags of ng_diag.flags */
#define NG_FLAG_NONFINITE 1u
#define NG_FLAG_RHO 2u      /* rho <= 0 somewhere */
#define NG_FLAG_P 4u        /* p <= 0 somewhere   */
#define NG_FLAG_DONE 8u     /* reached t_end or the step limit */

/* Gas of eqs. (1)-(7).  E_nue = rho * Cv * T (so C_k of eq. (8) is Cv / R);
 * tau = tau0 (rho/rho0)^tau_rho (T/T0)^tau_T, Q and I likewise (eq. (6));
 * (fx, fy) is the specific external force f of eqs. (2)-(3). */
typedef struct {
    double gamma, R, Cv;
    double rho0, T0;
    double tau0, tau_rho, tau_T;
    double Q0, Q_rho, Q_T;
    double I0, I_rho, I_T;
    double fx, fy;
} ng_gas;

/* Uniform grid of square cells of size h (section 2.3): ndim = 1 (ny = 1) or
 * 2; bc[4] = (x-low, x-high, y-low, y-high) boundary kinds NG_BC_* (y ends
 * ignored in 1D).  Planes are addressed with 32-bit byte offsets: at most
 * 2^30 cells in FP32 and 2^29 in FP64 and NG_MIXED.
 *
 * NG_BC_SOURCE (bc[0] only; bc[1] then must not be periodic): the two ghost
 * cells x = -h/2, -3h/2 hold, at the time t of the state a step starts from,
 * s = src_amp sin(omega t - k x) with k = 2 pi / src_lambda, omega = c k,
 *   rho = rho_b + s, u = (c / rho_b) s, v = 0, p = p_b + c^2 s,
 *   E_nu = E_nu,b + (E_nu,b / rho_b) s,
 * about the steady background at the reference point of eq. (6) (rho_b =
 * rho0, p_b = R rho0 T0, E_nu,b = rho0 Cv T0 + rho0 tau0 Q0, c = the frozen
 * sound speed sqrt(gamma p_b / rho_b)): a sound wave of wavelength
 * src_lambda entering the domain.  Requires src_lambda > 0 and |src_amp| <
 * rho_b / 2; both are ignored for other kinds.  In 2D, src_hw > 0 limits the
 * source to the ghost rows whose centre y has |y - src_yc| <= src_hw (the
 * other rows of that edge are free outflow); src_hw <= 0: the whole edge.
 *
 * Active wedge (2D sector run of section 3): wedge_tan > 0 confines the pump
 * and sink of eq. (6) (Q0, I0) to the cells whose centre has x >= wedge_x0
 * and |y - wedge_y0| <= (x - wedge_x0) wedge_tan; elsewhere the gas is
 * passive (Q = I = 0, relaxation only), and a source's background E_nu is the
 * passive one.  Requires a 2D grid and wedge_x0 >= 0.  wedge_tan <= 0: active
 * everywhere (the fields are ignored). */
typedef struct {
    int32_t ndim;
    int32_t reserved;
    int64_t nx, ny;
    double h;
    int32_t bc[4];
    double src_amp, src_lambda;
    double src_yc, src_hw;
    double wedge_x0, wedge_y0, wedge_tan;
} ng_grid;

/* cfl multiplies the bound of eq. (16); stiff_z is the dt/tau above which the
 * E_nu equation (4), relaxation and pump together, is integrated exactly over
 * the (half) step with E_nue, tau and Q frozen: E_nu relaxes toward
 * E_nue + tau rho Q by the factor exp(-dt/tau).  scheme: NG_MUSCL, or
 * NG_CSPH_TVD with a 1D grid, NG_FP64 and NG_HLL (any other combination, or
 * another value, is NG_EINVAL); with a forced source its three ghost
 * particles x = -h/2, -3h/2, -5h/2 carry the source's wave. */
typedef struct {
    double cfl;
    int32_t riemann;   /* NG_HLLC or NG_HLL */
    int32_t limiter;   /* NG_MINMOD         */
    int32_t precision; /* NG_FP64, NG_FP32 or NG_MIXED */
    int32_t scheme;    /* NG_MUSCL or NG_CSPH_TVD     */
    double stiff_z;
} ng_numerics;

/* Diagnostics.  total[] = h^d * sum over cells of (rho, rho u, rho v, E, E_nu)
 * accumulated in FP64 after the last step; src_budget[] = h^d * sum over steps
 * and cells of dt * Y_E (the rho (Q - I + v.f) row of Y in eq. (15)) and of the
 * E_nu source increment, so that total[3] - total0[3] = src_budget[0] and
 * total[4] - total0[4] = src_budget[1] up to rounding on periodic grids;
 * smax = max over cells of max(|v| + c, 2|v|) (eq. (16)) of the current state;
 * rho_min and p_min over cells of the current state. */
typedef struct {
    double t, dt_last, dt_next;
    int64_t steps;
    double total[5];
    double src_budget[2];
    double rho_min, p_min, smax;
    uint32_t flags;
    int32_t status;
} ng_diag;

typedef struct ng_solver ng_solver;
typedef struct ng_batch ng_batch;

const char* ng_strerror(int code);

/* ------------------------------------------------------------ one solve */

/* Device bytes that ng_init_state needs for this grid and precision: two state
 * buffers of (ndim + 3) planes plus per-step reduction space.  Returns NG_EINVAL
 * for an invalid grid. */
int ng_state_bytes(const ng_grid* grid, const ng_numerics* num, size_t* bytes);

/* Create a solver on caller-owned device memory and upload the initial state.
 *   prim:  host FP64 primitive planes (rho, u, [v], p, E_nu), layout above;
 *   t0:    initial time;
 *   dev_buf, dev_bytes: device memory of at least ng_state_bytes bytes,
 *          256-byte aligned;
 *   hip_stream: the stream every call of this solver enqueues on.
 * Validates gamma > 1, R > 0, h > 0, n >= 4 per dimension, 0 < cfl < 1,
 * tau0 > 0, and rho > 0, p > 0 and finite values in prim (NG_EINVAL);
 * dev_bytes too small gives NG_ENOMEM.  Synchronising (computes the first dt
 * and the initial totals). */
int ng_init_state(const ng_gas* gas, const ng_grid* grid, const ng_numerics* num,
                  const double* prim, double t0, void* dev_buf, size_t dev_bytes,
                  void* hip_stream, ng_solver** out);

/* Same from conserved planes (rho, rho u, [rho v], E, E_nu). */
int ng_init_conserved(const ng_gas* gas, const ng_grid* grid, const ng_numerics* num,
                      const double* cons, double t0, void* dev_buf, size_t dev_bytes,
                      void* hip_stream, ng_solver** out);

/* Enqueue nsteps steps of eq. (15), each with dt from eq. (16) evaluated on the
 * state it starts from (no end time).  Asynchronous. */
int ng_step(ng_solver* s, int64_t nsteps);

/* Advance until t_end (the last dt is shortened to land on it) or until
 * max_steps more steps, whichever comes first; steps run as captured HIP
 * graphs whose kernels read t, dt and the stop condition from device memory.
 * Synchronising; *steps_taken (may be NULL) receives the steps done. */
int ng_run_to_time(ng_solver* s, double t_end, int64_t max_steps, int64_t* steps_taken);

/* Diagnostics of the current state.  Synchronising. */
int ng_diagnostics(ng_solver* s, ng_diag* out);

/* Read the current state as FP64 primitive / conserved planes (whatever the
 * run precision).  Synchronising. */
int ng_get_state(ng_solver* s, double* prim_out);
int ng_get_conserved(ng_solver* s, double* cons_out);

/* Launch shape of the step kernel: rows per work item (2D) or 60-cell
 * segments per work item (1D), and waves per workgroup.  Results do not
 * depend on it (every cell's arithmetic is the same); only the order of the
 * FP64 total sums does.  0 keeps the current value; -1 (the default)
 * chooses from the solves launched together (all big solves of the dim):
 * 2D the largest of 32, 24, 16, 12, 8, 6 and 4 rows at which their work
 * items (one wavefront each) add up to at least 2304, else 4; 1D 8 segments
 * if they give 8192 work items, else the largest of 4, 2 and 1 reaching
 * 1024, else 1.  A lone grid smaller than 4096^2 so keeps the SIMDs busy; a
 * batch with work enough keeps long chunks.  Waves per workgroup 1, 2 or 4,
 * or -1: 4, except 2 for a 1D launch of fewer than 2048 work items (default
 * -1 in 1D, 4 in 2D).  2D rows below 4 and other values: EINVAL. */
int ng_set_launch(ng_solver* s, int32_t rows_per_item, int32_t waves_per_block);

/* Steps per captured graph (default 64, 1 to 4096): calls of ng_step and
 * ng_run_to_time replay whole graphs of this many steps and launch the rest
 * directly.  Waits for the steps in flight when a graph exists.  EINVAL
 * outside 1..4096. */
int ng_set_graph_steps(ng_solver* s, int32_t steps);

/* Solves of at most max_cells cells are advanced by a persistent kernel in
 * which one workgroup runs many steps per launch (no launch or host round trip
 * per step); larger ones take one launch per step over the whole GPU.  -1
 * restores the default (4096 cells in FP32, 2048 in FP64), 0 turns the
 * persistent path off.  Both paths give bitwise the same state. */
int ng_set_small_limit(ng_solver* s, int64_t max_cells);

/* Cooperative path (the time loop of eq. (15) with the dt of eq. (16) chosen
 * after every step).  A solve that is alone in its object, 1D and of at most
 * max_cells cells is advanced by one cooperative launch per call (up to 65536
 * steps each): every step, its workgroups -- all resident together -- update
 * their segments, publish their largest signal speed and failure flags in
 * device memory, and each reads those of all the others and accepts or
 * rejects the step and takes the next dt alike (a forced source's ghosts
 * follow its own t).  No launch or host round trip per step; the state, t
 * and dt are bitwise those of one launch per step (only the summation order
 * of the FP64 totals differs).
 * max_cells: -1 restores the default (4194304), 0 turns the path off (the
 * persistent one-workgroup path or one launch per step take over).
 * spin_limit: polls of memory (about a microsecond each) a workgroup spends
 * in one barrier wait before it gives up (-1: the default, 1048576); a wait
 * that runs out ends the launch early with every kernel exiting, and the
 * next synchronising call reports NG_ESTALL.  Cooperative launches must be
 * supported by the device (else the other paths run).  Synchronising;
 * NG_EINVAL for values below -1. */
int ng_set_coop(ng_solver* s, int64_t max_cells, int32_t spin_limit);

/* Step acceptance inside the step kernel (1, default) or by a separate
 * kernel (0); see ng_batch_set_fused_accept. */
int ng_set_fused_accept(ng_solver* s, int32_t on);

/* Kernel timing: ng_enable_timing(s, nsteps, every) with nsteps > 0 makes
 * later ng_step calls launch each step directly (no graph).  The step and
 * finalize kernels of steps every-1, 2*every-1, ... and of the last step of
 * each call (counting from 0) record their own start and end in HIP events
 * (the launch carries the events, so no event packets sit between the
 * kernels); the other steps launch without events.  every >= 1: 1 times every
 * step, a larger stride keeps the cost of the timed launches (a few
 * microseconds each) out of the run's total.  The events for nsteps steps are
 * created here, outside any timed region; nsteps 0 turns timing off.  EINVAL
 * for nsteps < 0 or every < 1.
 * ng_kernel_time returns the mean kernel durations in milliseconds over the
 * timed launches of the last timed ng_step call (finalize_ms 0 when the step
 * kernel accepted its own steps) and the number of step launches timed. */
int ng_enable_timing(ng_solver* s, int32_t nsteps, int32_t every);
int ng_kernel_time(ng_solver* s, double* step_ms, double* finalize_ms, int64_t* launches);

const char* ng_last_error(const ng_solver* s);

/* For callers that cannot allocate memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): one step of eq. (15)
 * (or, with num->scheme = NG_CSPH_TVD, one CSPH-TVD step of section 2.3) on an
 * FP64 state in caller device memory, calling no hipMalloc, hipFree or
 * other allocating routine.  Its scratch -- the solve's descriptor and control
 * block, the workgroup table and the per-workgroup reduction records -- lives
 * in a static device array of 2 MiB that each GPU the library runs on holds
 * until the process ends; a grid whose launch needs more (about 20000
 * workgroups, e.g. beyond 8192^2 cells in 2D) is refused with NG_ENOMEM.
 *   gas, grid, num: as for ng_init_state; num->precision must be NG_FP64;
 *   U_in:  device, FP64 conserved planes (rho, rho u, [rho v], E, E_nu) in the
 *          layout of the host arrays, the state at time t (read only);
 *   U_out: device, same size, distinct from U_in: receives the state after
 *          the step (undefined if the call returns NG_EPHYS);
 *   t, t_end: time of U_in and end time (the step is shortened to land on
 *          t_end > t; t_end <= t: no end time); dt is that of eq. (16) on U_in;
 *   hip_stream: the stream the kernels are enqueued on;
 *   out:   NULL (the call only enqueues: asynchronous, usable under stream
 *          capture) or a host ng_diag that receives t, dt_last, the totals of
 *          U_out, ... (synchronises the stream; returns NG_EPHYS when the step
 *          was rejected).
 * The state is bitwise that of ng_init_conserved(U_in) + ng_step(1).  Every
 * call on a GPU shares that GPU's scratch (each call writes all of it that it
 * reads): calls that overlap on one GPU race, so enqueue them on one stream.
 * Errors: NG_EINVAL (invalid arguments, as ng_init_state, or another
 * precision), NG_ENOMEM (grid beyond the scratch), NG_EDEVICE; the text is
 * returned by ng_static_last_error (per host thread). */
int ng_step_static(const ng_gas* gas, const ng_grid* grid, const ng_numerics* num,
                   const void* U_in, void* U_out, double t, double t_end, void* hip_stream,
                   ng_diag* out);
const char* ng_static_last_error(void);

/* Free the host-side object.  Never frees dev_buf or the stream. */
void ng_destroy(ng_solver* s);

/* ------------------------------------------------- batches of many solves */
/*
 * A batch advances many independent solves of one precision -- any mix of 1D
 * and 2D grids, sizes and gas parameters -- with one step kernel per dimension
 * per step, each solve with its own dt, t, end time and totals.  Every solve's
 * arithmetic is the same as when it runs alone, so its results do not depend
 * on the batch composition.  Solves live in a caller-owned device arena; the
 * batch sub-allocates it.
 */

/* capacity: maximum number of live solves; precision: NG_FP32, NG_FP64 or NG_MIXED;
 * dev_buf/dev_bytes: the arena (256-byte aligned). */
int ng_batch_create(int32_t capacity, int32_t precision, void* dev_buf, size_t dev_bytes,
                    void* hip_stream, ng_batch** out);

/* Device bytes one solve of this grid occupies in a batch arena. */
int ng_batch_solve_bytes(const ng_grid* grid, int32_t precision, size_t* bytes);

/* *fits = 1 if a solve of this grid would find a free slot and a free block
 * of ng_batch_solve_bytes() in the arena now, else 0 (a caller can defer
 * preparing the initial state of a solve that cannot be added yet).
 * NG_EINVAL on a null pointer or a grid that is not 1D or 2D. */
int ng_batch_fits(const ng_batch* b, const ng_grid* grid, int32_t* fits);

/* Add a solve (validation as ng_init_state; num->precision must match the
 * batch).  It runs until t_end (> t0) or max_steps steps.  *slot receives its
 * slot number.  NG_EFULL when no slot or arena space is free; NG_EINVAL when a
 * cell of the initial state is non-finite or has rho <= 0 or p <= 0.
 * Does not wait for steps in flight: the host converts and checks `prim`
 * while they run, the upload runs on a second stream of the library, and the
 * solve's priming pass is ordered on the batch stream behind it; the solve
 * joins the next ng_batch_run.  `prim` may be reused on return.  A state that
 * the device check rejects shows as NG_EPHYS in its diagnostics. */
int ng_batch_add(ng_batch* b, const ng_gas* gas, const ng_grid* grid, const ng_numerics* num,
                 const double* prim, double t0, double t_end, int64_t max_steps,
                 int32_t* slot);

/* Enqueue nsteps steps of every unfinished solve (finished ones are skipped on
 * the device).  Asynchronous. */
int ng_batch_run(ng_batch* b, int64_t nsteps);

/* Wait for the stream and list up to cap slots whose solve has finished
 * (reached t_end or max_steps, or failed) and not yet been reported.
 * Synchronising. */
int ng_batch_poll(ng_batch* b, int32_t* done_slots, int32_t cap, int32_t* ndone);

/* Number of live solves that have not finished.  Synchronising. */
int ng_batch_active(ng_batch* b, int32_t* nactive);

int ng_batch_diagnostics(ng_batch* b, int32_t slot, ng_diag* out);
int ng_batch_get_state(ng_batch* b, int32_t slot, double* prim_out);
int ng_batch_get_conserved(ng_batch* b, int32_t slot, double* cons_out);

/* Release a slot and its arena space. */
int ng_batch_remove(ng_batch* b, int32_t slot);

/* How a step is accepted (dt, t and totals advanced): on = 1 (default) lets
 * solves of up to 256 step workgroups be accepted by the last workgroup of the
 * step kernel itself (one launch per step); larger solves, and all solves when
 * on = 0, are accepted by a separate one-workgroup kernel after the step.
 * The state, t and dt are identical either way. */
int ng_batch_set_fused_accept(ng_batch* b, int32_t on);

/* Persistent-path size limit of a batch (see ng_set_small_limit). */
int ng_batch_set_small_limit(ng_batch* b, int64_t max_cells);

/* Cooperative path of a batch (see ng_set_coop): taken only while the batch
 * holds exactly one live solve that qualifies. */
int ng_batch_set_coop(ng_batch* b, int64_t max_cells, int32_t spin_limit);

/* Launch shape of the batched step kernels (see ng_set_launch). */
int ng_batch_set_launch(ng_batch* b, int32_t dim, int32_t rows_per_item,
                        int32_t waves_per_block);

const char* ng_batch_last_error(const ng_batch* b);
void ng_batch_destroy(ng_batch* b);

#ifdef __cplusplus
}
#endif
#endif /* NG_H */
