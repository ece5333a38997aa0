/*
 * hydro.h -- C ABI of the MI355X library for the directionally split,
 * second-order Godunov sweep of the 2D compressible Euler equations.
 *
 * The problem is the one the paper states (Section 1): a fixed rectangular 2D
 * domain, the compressible Euler equations of an ideal gas, a finite-volume
 * discretisation, and a second-order Godunov scheme with directional
 * splitting -- one 1D update per direction, performed successively, each
 * solving a Riemann problem at every cell interface and updating the cells
 * from the interface fluxes.  A 1D update of cell i reads cells i-2..i+2 of
 * its pencil only (Figures 1 and 2); per pencil the work is READ, COMPUTE
 * (primitive variables, Riemann problems, incoming fluxes), WRITE
 * (Figure 5), with boundary conditions applied in every time step.
 *
 * Numerical readings (the paper delegates the details to its references):
 * minmod-limited slopes of (rho, u_n, u_t, p); MUSCL-Hancock half-step trace;
 * star pressure by Newton on the two-shock wave function from the
 * two-rarefaction guess, stopped at |dp| <= tol*p or after niter iterations;
 * linear sampling across rarefaction fans; CFL time step
 * dt = cfl * h / max(|u|+c, |v|+c); floors rho >= 1e-10, c >= 1e-10; x-sweep
 * then y-sweep every step.  Options (hydro_options_t) select the MC or van
 * Leer limiter, an alternating sweep order, the exact Riemann solver or the
 * HLLC flux; hydro_set_scalars adds passive scalars.
 *
 * STATE LAYOUT.  U is a caller-owned device array [4 + ns][ny][pitch] of
 * float64 (HYDRO_F64) or float32 (HYDRO_F32): planes rho, rho*u, rho*v, E,
 * then rho*X for each of the ns passive scalars X (hydro_set_scalars; 0 by
 * default); x is the fastest index, pitch >= nx elements (a multiple of 64
 * keeps rows aligned).
 * Interior cells only: ghost cells never live in user memory.  Cells are
 * square, h = 1 / max(nx, ny).  The library never frees caller memory.
 * Sweeps are out of place: the handle owns a second buffer of the same size
 * (allocated by hydro_bind); the first sweep of a step writes it, the second
 * writes U back, and a lone hydro_sweep copies its result back, so after
 * every call U holds the current state.
 *
 * ERRORS.  Every call returns HYDRO_OK (0) or a negative code and sets a
 * thread-local message (hydro_last_error).  No call aborts or throws.
 * HIP failures map to HYDRO_EDEVICE.  Non-physical states met by a sweep
 * (non-finite values, rho <= 0) are latched on the device and reported as
 * HYDRO_ENONPHYS by the next call that synchronises.
 *
 * NAMES.  The five calls the method needs are hydro_create, hydro_compute_dt,
 * hydro_sweep, hydro_step and hydro_conserved_totals.  Three calls around them
 * differ from the first sketch of this interface:
 *   - hydro_batch_layout replaces a call that returned only the batch
 *     buffer's element count; it also returns each grid's offset and pitch.
 *   - hydro_mlp_grad replaces a separate backward call: it fuses the forward
 *     pass, the loss and the backward pass, so activations never reach memory.
 *   - The network and its gradient are a packed device buffer (void *) and a
 *     flat float array, not C structs.  Adam's settings are plain arguments.
 *
 * STREAMS.  All device work of a handle runs on the stream given to
 * hydro_bind, in order.  hydro_sweep and hydro_step never synchronise and
 * keep dt on the device, so they can be captured into a HIP graph;
 * hydro_compute_dt, hydro_conserved_totals, hydro_get_clock and
 * hydro_riemann_stats synchronise that stream.  A handle is not thread-safe;
 * separate handles are independent.
 */
#ifndef HYDRO_H
#define HYDRO_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hydro_s hydro_t;

enum { HYDRO_BC_REFLECT = 1, HYDRO_BC_OUTFLOW = 2, HYDRO_BC_PERIODIC = 3 };
enum { HYDRO_DIR_X = 0, HYDRO_DIR_Y = 1 };
enum { HYDRO_F64 = 0, HYDRO_F32 = 1 };
enum { HYDRO_GUESS_PTR = 0, HYDRO_GUESS_MLP = 1 };
enum {
  HYDRO_OK = 0,
  HYDRO_EINVAL = -1,   /* bad argument                                   */
  HYDRO_ENOMEM = -2,   /* device allocation failed                       */
  HYDRO_EDEVICE = -3,  /* HIP runtime error                              */
  HYDRO_ENONPHYS = -4, /* a sweep produced a non-physical state          */
  HYDRO_ESTATE = -5    /* call not valid in the handle's state (unbound) */
};

#define HYDRO_MAX_NITER 32
#define HYDRO_MAX_SCALARS 1

#define HYDRO_LEARNED_GATE_DEFAULT 1.0

/* Slope limiters (options.limiter): minmod (default); MC, the monotonized
 * central sign(a) min(2|a|, 2|b|, |a+b|/2); van Leer's harmonic mean
 * 2ab/(a+b); all 0 unless both one-sided differences a, b share a sign. */
enum { HYDRO_LIMITER_MINMOD = 0, HYDRO_LIMITER_MC = 1, HYDRO_LIMITER_VANLEER = 2 };
/* Sweep order (options.order): x then y every step (default), or x then y
 * on even steps and y then x on odd steps (by the handle's step count). */
enum { HYDRO_ORDER_XY = 0, HYDRO_ORDER_ALTERNATE = 1 };
/* Interface solver (options.riemann).  The paper delegates its Riemann
 * solver to a reference (Section 1); the default reading is the two-shock
 * solver, Newton from the two-rarefaction guess.  HYDRO_RIEMANN_EXACT: the
 * exact Riemann solver, Newton on the exact shock and rarefaction curves from
 * the same guess with the same cap, test and floors, then the exact
 * self-similar state at x/t = 0 (rarefaction fans included).
 * HYDRO_RIEMANN_HLLC: the HLLC flux with Einfeldt's wave bounds from Roe
 * averages; no iteration, so Riemann statistics and the interface logger
 * record nothing and the learned guess is rejected (HYDRO_EINVAL). */
enum { HYDRO_RIEMANN_TWO_SHOCK = 0, HYDRO_RIEMANN_EXACT = 1, HYDRO_RIEMANN_HLLC = 2 };
/* Form of the y-sweep kernel (options.ysweep); same numerics, results equal
 * to rounding.  HYDRO_YSWEEP_MARCH (default): each thread marches down one
 * column with the 5-cell stencil in registers, 64 adjacent columns per wave,
 * so every load and store is one coalesced row access.  HYDRO_YSWEEP_TILE:
 * 16-column by 64-row tiles are read row-coalesced into LDS, transposed, and
 * swept one cell per lane with the x-sweep's code (a pencil tile staged in
 * LDS with its two ghost cells per side); slower on MI355X (more
 * instructions per cell for a kernel bound by instruction issue). */
enum { HYDRO_YSWEEP_MARCH = 0, HYDRO_YSWEEP_TILE = 1 };

/* Solver options (hydro_set_options).  Defaults: niter 10, tol 1e-8,
 * guess HYDRO_GUESS_PTR, stats 0, tiles chosen by the library,
 * learned_gate HYDRO_LEARNED_GATE_DEFAULT, limiter HYDRO_LIMITER_MINMOD,
 * order HYDRO_ORDER_XY, riemann HYDRO_RIEMANN_TWO_SHOCK,
 * ysweep HYDRO_YSWEEP_MARCH. */
typedef struct {
  int niter;     /* Newton iteration cap, 1..HYDRO_MAX_NITER              */
  double tol;    /* convergence test |dp| <= tol * p, > 0                  */
  int guess;     /* HYDRO_GUESS_PTR or HYDRO_GUESS_MLP (needs hydro_set_mlp)*/
  int stats;     /* nonzero: count Newton iterations per interface         */
  int seg_x;     /* x-sweep: consecutive 60-cell wave segments per wave;
                    0 = library default (8; hydro_autotune picks among
                    1, 2, 4, 8, 16).  Results do not depend on it.          */
  int seg_y;     /* y-sweep: cells per marching thread; 0 = default (128);
                    results do not depend on it                            */
  double learned_gate; /* with HYDRO_GUESS_MLP: strength s above which an
                    interface takes the learned guess; the others keep the
                    two-rarefaction guess, and a wave evaluates the network
                    only when one of its interfaces is above.  An interface
                    is above when max(pL,pR) > e^s min(pL,pR) or
                    (uR-uL)^2 (rhoL+rhoR) > s^2 gamma (pL+pR).  s <= 0: every
                    interface takes the learned guess.  Finite, <= 50.     */
  int limiter;   /* HYDRO_LIMITER_*                                        */
  int order;     /* HYDRO_ORDER_*                                          */
  int riemann;   /* HYDRO_RIEMANN_*                                        */
  int ysweep;    /* HYDRO_YSWEEP_*                                         */
} hydro_options_t;

/* Riemann-solver statistics accumulated since the last reset
 * (hydro_riemann_stats).  Collected only while options.stats != 0. */
typedef struct {
  long long interfaces;                  /* Riemann problems solved         */
  long long hist[HYDRO_MAX_NITER + 1];   /* hist[k]: converged after k
                                            iterations; hist[0]: iteration
                                            cap reached unconverged;
                                            hist[HYDRO_MAX_NITER] also holds
                                            longer counts (a failed learned
                                            start adds up to 4 to the cap)  */
  long long fallbacks;                   /* learned guess rejected          */
  long long wave_hist[HYDRO_MAX_NITER + 1]; /* groups of interfaces a wave
                                            solves together (up to 64) by
                                            their largest iteration count
                                            (the cap for an unconverged one):
                                            the wave runs that many          */
} hydro_stats_t;

/* Launch shape chosen by the autotuner (hydro_autotune / hydro_batch_autotune).
 * Results never depend on it. */
typedef struct {
  int seg_x;          /* x-sweep: 60-cell segments per wave item                 */
  int seg_y;          /* y-sweep: rows marched per wave item                     */
  unsigned blocks_x;  /* 0: one 4-wave block per 4 items; else persistent blocks */
  unsigned blocks_y;
  double ms_x, ms_y;  /* best measured sweep times (ms); -1 when reused          */
  int candidates;     /* launch shapes timed                                     */
  int cached;         /* 1: reused an earlier tuning of the same grid shapes     */
} hydro_tune_t;

/* Paper, Section 1 (the problem: a fixed rectangular 2D domain, the
 * compressible Euler equations of an ideal gas, finite volumes) and Figure 5
 * (boundary conditions applied every step).
 * Create a solver for an nx x ny grid (both >= 2) of an ideal gas with ratio
 * of specific heats gamma > 1, Courant number 0 < cfl <= 1 and boundary type
 * bc (one of HYDRO_BC_*, applied on all four sides).  Allocates the handle's
 * small device scratch on the current HIP device.  Returns NULL on error
 * (hydro_last_error gives the reason). */
hydro_t *hydro_create(int nx, int ny, double gamma, double cfl, int bc);

/* Release the handle and its scratch (never the bound state). NULL is a no-op. */
void hydro_destroy(hydro_t *h);

/* Message of the last failed call on this thread ("" if none). */
const char *hydro_last_error(void);

/* Carry n passive scalars (0..HYDRO_MAX_SCALARS): quantities X advected with
 * the flow and conserved as rho X, stored after E.  Each is reconstructed
 * like the primitive variables (same limiter, MUSCL-Hancock faces with the
 * advective source -u dX) and crosses an interface with the mass flux, at the
 * value of the side of the contact that holds x/t = 0.  They do not act on
 * the flow.  Only before hydro_bind (HYDRO_ESTATE after). */
int hydro_set_scalars(hydro_t *h, int n);

/* Paper, Figure 5 (U(i,j), the 2D buffer of conservative variables that every
 * sweep reads and writes back).
 * Bind the state U (device pointer, layout above, pitch in elements) of type
 * dtype and the HIP stream (hipStream_t; NULL = default stream) all later
 * work runs on.  Rebinding is allowed; it invalidates the fused max speed, so
 * the next step recomputes dt from U.  Call it again (or hydro_invalidate)
 * after modifying U outside the library. */
int hydro_bind(hydro_t *h, void *U, long pitch, int dtype, void *hip_stream);

/* Forget the max wave speed fused into the last step's second sweep (U
 * changed outside the library). */
int hydro_invalidate(hydro_t *h);

/* Paper, Section 1 (the limiter, the Riemann solver [4] and the scheme [5]
 * are delegated to references): the readings and options of hydro_options_t.
 * Set or read the solver options of a handle; a change drops any captured
 * graph.  Invalid values return HYDRO_EINVAL and leave the options as they
 * were. */
int hydro_set_options(hydro_t *h, const hydro_options_t *o);
int hydro_get_options(const hydro_t *h, hydro_options_t *o);

/* Paper, Figure 5 (one dt per time step n, shared by both directional
 * sweeps); the paper does not give the formula, and the CFL bound below is
 * the reading taken.
 * Time step from the bound state: dt = cfl * h / max over cells of
 * max(|u|+c, |v|+c).  Stores dt on the device for later sweeps and returns
 * it (> 0), or a negative error code.  Synchronises the stream. */
double hydro_compute_dt(hydro_t *h);

/* Paper, Section 1 (a one-dimensional second-order Godunov update along one
 * direction, a Riemann problem at every interface), Figures 1 and 2 (cell i
 * reads cells i-2..i+2 of its pencil only) and Figure 5 (per pencil READ,
 * COMPUTE: primitive variables, Riemann problems, incoming fluxes, WRITE).
 * One directional sweep (HYDRO_DIR_X: rows, HYDRO_DIR_Y: columns) of the
 * bound state with the stored dt, boundary conditions applied along that
 * direction (two ghost cells per side).  Asynchronous.  Does not advance the
 * clock. */
int hydro_sweep(hydro_t *h, int dir);

/* Paper, Section 1 (directional splitting: at each time step the 1D scheme
 * runs along each direction in turn) and Figure 5 (boundary conditions, the
 * loop over one direction's pencils, then the other's).
 * One time step: dt from the current state (taken from the max wave speed
 * fused into the previous step's second sweep when still valid, otherwise
 * from a reduction over U), then the x-sweep and the y-sweep (with
 * HYDRO_ORDER_ALTERNATE: the y-sweep first on odd steps), both with that dt;
 * t += dt, step += 1 on the device.  Asynchronous, no host synchronisation. */
int hydro_step(hydro_t *h);

/* Paper, Section 1 (finite-volume form of the Euler equations: cell values
 * are averages of conserved quantities, so their sums times the cell area
 * are the domain's mass, momentum and energy).
 * out[k] = sum over cells of U_k * h^2 (k = rho, rho u, rho v, E, then the
 * passive scalars' rho X: 4 + ns values), summed in FP64 in a fixed order
 * (deterministic), also for float32 states.  Synchronises the stream. */
int hydro_conserved_totals(hydro_t *h, double *out);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 * One time step of hydro_step (dt from the max wave speed of U, then the
 * x-sweep and the y-sweep with that dt) for n independent grids held in
 * caller buffers, with no handle and no device allocation: the per-grid
 * descriptors and device state the kernels need live in a static device
 * array inside the library (one copy per GPU, about 12 KB, held until the
 * process ends), resolved on the first call on each device.  Default
 * options (minmod, two-shock solver, Newton cap 10, tol 1e-8, two-rarefaction
 * guess, x then y) and the default launch shape; no clock, statistics,
 * passive scalars or learned guess.
 *   n                  1..HYDRO_NOALLOC_MAX_GRIDS grids (more: HYDRO_EINVAL,
 *                      the size of the static array)
 *   nx, ny, bc         host arrays [n]: grid sides (>= 2) and HYDRO_BC_*
 *   offsets, pitches   host arrays [n]: element offset of grid g's plane 0
 *                      and its row pitch (>= nx[g]); grid g occupies
 *                      [offsets[g], offsets[g] + 4 ny[g] pitches[g]) of each
 *                      buffer in the layout of a single grid; grids must not
 *                      overlap
 *   dtype              HYDRO_F64 or HYDRO_F32, all three buffers
 *   U                  device, input: the state at the start of the step
 *   U_half             device, output: the state after the x-sweep; must not
 *                      overlap U or U_out
 *   U_out              device, output: the state after the step; may be U
 *                      itself (in-place step), else must not overlap it
 *   dt_out             device array [n] or NULL, output: the dt grid g
 *                      advanced by, NaN if a sweep of grid g produced a
 *                      non-physical state
 *   hip_stream         hipStream_t the work is enqueued on (NULL: default)
 * All buffers are caller-owned.  Asynchronous: returns after enqueueing (no
 * synchronisation), HYDRO_EINVAL for bad arguments, HYDRO_EDEVICE for a HIP
 * error.  Every call on one GPU reuses that GPU's static array: calls that
 * overlap in time on one GPU (other streams or host threads) race and must
 * be serialised by the caller. */
#define HYDRO_NOALLOC_MAX_GRIDS 16
int hydro_step_noalloc(int n, const int *nx, const int *ny, const int *bc,
                       const long long *offsets, const long *pitches, int dtype, double gamma,
                       double cfl, const void *U, void *U_half, void *U_out, double *dt_out,
                       void *hip_stream);

/* Simulated time, steps taken and the last dt (device clock).  Synchronises. */
int hydro_get_clock(hydro_t *h, double *t, long *step, double *dt);
/* Set the device clock (checkpoint restart); dt is kept.  Asynchronous. */
int hydro_set_clock(hydro_t *h, double t, long step);

/* Paper, Figure 5 (the loop over time steps n), as one captured unit.
 * Advance nsteps time steps by replaying a HIP graph of nsteps consecutive
 * hydro_step calls, captured on the bound stream at the first call (and again
 * after hydro_bind, hydro_set_options or a different nsteps).  The bound
 * stream must not be the legacy default stream (capture is not allowed
 * there).  Results are bitwise those of nsteps hydro_step calls.
 * Asynchronous.  nsteps in 1..4096. */
int hydro_graph_steps(hydro_t *h, int nsteps);

/* Copy the Riemann statistics (synchronises); reset clears them. */
int hydro_riemann_stats(hydro_t *h, hydro_stats_t *s, int reset);

/* Time candidate launch shapes of both sweeps on the bound state and keep
 * the fastest: segments per work item (for the y-sweep also lengths whose
 * items fill whole rounds of the resident waves) times persistent block
 * counts; the three fastest are re-timed and the lowest median wins.  U is
 * not modified; the fused max speed is invalidated.  use_cache reuses the
 * result of an earlier tuning of the same grid shapes, dtype, starting guess,
 * limiter and solver in this process.  Synchronises.  out may be NULL. */
int hydro_autotune(hydro_t *h, hydro_tune_t *out, int use_cache);

/* Kernel timing.  While enabled, hydro_step records a HIP event pair on the
 * bound stream around each of its phases (dt, x-sweep, y-sweep), except
 * under stream capture.  hydro_get_profile synchronises, returns the summed
 * durations in milliseconds and launch counts per phase since the last
 * reset, and optionally resets them. */
enum { HYDRO_PHASE_DT = 0, HYDRO_PHASE_SWEEP_X = 1, HYDRO_PHASE_SWEEP_Y = 2, HYDRO_NPHASES = 3 };
int hydro_set_profiling(hydro_t *h, int enable);
int hydro_get_profile(hydro_t *h, double ms[HYDRO_NPHASES], long long launches[HYDRO_NPHASES],
                      int reset);

/* ------------------------------------------------------------------------
 * Learned starting guess for the star pressure (an addition to the paper's
 * method; the two-rarefaction guess with the full Newton cap stays the
 * fallback).  A 6 -> 32 -> 32 -> 1 network with ReLU activations, BF16 weights
 * and activations on the MFMA units, FP32 accumulation.  It corrects the
 * two-rarefaction guess p_ptr.  Features of an interface:
 * a = ln(rho_L/rho_bar), b = ln(p_L/p_bar), w = asinh((u_L-u_bar)/c_bar),
 * q = ln(p_ptr/p_bar), x = (a, b, w, q, -a, -b) with geometric means rho_bar,
 * p_bar, u_bar the mean velocity and c_bar = sqrt(gamma p_bar/rho_bar);
 * output y ~ ln(p_star / p_ptr).  In a sweep with options.guess =
 * HYDRO_GUESS_MLP, Newton runs at most 4 iterations from p_ptr exp(y); if its
 * convergence test fails (or the guess is not a finite positive pressure) the
 * interface restarts from p_ptr with the full cap and counts as a fallback.
 *
 * Parameters: HYDRO_MLP_PARAMS FP32 values, flat and row-major:
 * W1[32][6], b1[32], W2[32][32], b2[32], W3[32], b3.  All pointers below are
 * device memory owned by the caller; all calls are asynchronous on `stream`.
 * ------------------------------------------------------------------------ */
#define HYDRO_MLP_PARAMS 1313

/* Bytes of the packed device network (BF16 weights in MFMA lane order). */
size_t hydro_mlp_dev_bytes(void);
/* Pack FP32 parameters into a device network (and mark it invalid if any
 * parameter is not finite: then every learned guess falls back). */
int hydro_mlp_pack(const float *params, void *mlp, void *stream);
/* Logged interface records [n][8] -> features X [n][6] and targets
 * Y [n] = ln(p_star / p_ptr) (Y may be NULL); p_ptr is the two-rarefaction
 * guess of the record's states, in FP64. */
int hydro_mlp_features(const float *records, long long n, double gamma, float *X, float *Y,
                       void *stream);
/* Y[n] = network output for X [n][6]. */
int hydro_mlp_forward(const void *mlp, const float *X, float *Y, long long n, void *stream);
/* Gradient of the mean squared error (1/n) sum (y - T)^2 with respect to the
 * parameters (grad[HYDRO_MLP_PARAMS], overwritten) and the loss (may be NULL),
 * using scratch of hydro_mlp_grad_scratch_bytes(n). */
size_t hydro_mlp_grad_scratch_bytes(long long n);
int hydro_mlp_grad(const void *mlp, const float *X, const float *T, long long n, float *scratch,
                   float *grad, float *loss, void *stream);
/* One Adam step (step >= 1 for the bias correction) on FP32 master
 * parameters with moment buffers m, v; repack with hydro_mlp_pack after. */
int hydro_mlp_adam(float *params, float *m, float *v, const float *grad, long long step,
                   double lr, double beta1, double beta2, double eps, void *stream);
/* Use a packed network (borrowed; NULL detaches it) for HYDRO_GUESS_MLP. */
int hydro_set_mlp(hydro_t *h, const void *mlp);
/* Interface-state logger: while records != NULL, every sweep offers each
 * interface with probability rate_smooth (rate_strong when the jump
 * |ln(p_L/p_R)| + |u_R-u_L|/c_bar exceeds 0.05) and appends
 * (rho_L, u_L, p_L, rho_R, u_R, p_R, p*, jump) as 8 floats until capacity
 * records are stored.  Seeded hash per (grid, step, interface, direction). */
int hydro_set_logger(hydro_t *h, float *records, long long capacity, unsigned long long seed,
                     double rate_smooth, double rate_strong);
/* Records offered so far (stored: min(count, capacity)); synchronises. */
long long hydro_logger_count(hydro_t *h);

/* ------------------------------------------------------------------------
 * Batches: n independent grids of uneven sizes advanced together, one kernel
 * launch per sweep over all of them (persistent wave loop over a work list
 * of (grid, segment) items), each grid with its own dt, clock and status.
 * Same numerics and readings as a single grid.
 *
 * LAYOUT.  All grids live in one caller-owned device buffer; grid g occupies
 * [offsets[g], offsets[g] + (4 + ns) * ny[g] * pitches[g]) elements with the
 * layout of a single grid ([4 + ns][ny][pitch], x fastest; ns passive
 * scalars, hydro_batch_set_scalars).  hydro_batch_layout gives the
 * offsets and pitches the library uses (rows padded to 256 bytes).
 * ------------------------------------------------------------------------ */
typedef struct hydro_batch_s hydro_batch_t;

/* n >= 1 grids; nx[g], ny[g] >= 2; bc[g] one of HYDRO_BC_*; NULL on error. */
hydro_batch_t *hydro_batch_create(int n, const int *nx, const int *ny, double gamma,
                                  double cfl, const int *bc);
void hydro_batch_destroy(hydro_batch_t *b);
/* Returns the elements per state buffer for dtype and fills offsets[n] and
 * pitches[n] (either may be NULL); negative on error. */
long long hydro_batch_layout(const hydro_batch_t *b, int dtype, long long *offsets,
                             long *pitches);
/* Bind the packed state (layout above) and stream; allocates the second
 * buffer. */
int hydro_batch_bind(hydro_batch_t *b, void *U, int dtype, void *hip_stream);
int hydro_batch_set_options(hydro_batch_t *b, const hydro_options_t *o);
/* Passive scalars of every grid, as hydro_set_scalars: before binding (and
 * before hydro_batch_layout, whose sizes include them). */
int hydro_batch_set_scalars(hydro_batch_t *b, int n);
int hydro_batch_invalidate(hydro_batch_t *b);
/* Per-grid dt into dt[n] (may be NULL); synchronises. */
int hydro_batch_compute_dt(hydro_batch_t *b, double *dt);
/* One time step of every grid (its own dt); asynchronous. */
int hydro_batch_step(hydro_batch_t *b);
/* nsteps steps of every grid as one replay of a captured HIP graph. */
int hydro_batch_graph_steps(hydro_batch_t *b, int nsteps);
/* out[(4 + ns) g + k]: totals of grid g; synchronises. */
int hydro_batch_totals(hydro_batch_t *b, double *out);
/* Per-grid clocks (arrays of n, any may be NULL); synchronises. */
int hydro_batch_get_clock(hydro_batch_t *b, double *t, long *step, double *dt);
/* Riemann statistics summed over the grids; synchronises. */
int hydro_batch_riemann_stats(hydro_batch_t *b, hydro_stats_t *s, int reset);
int hydro_batch_autotune(hydro_batch_t *b, hydro_tune_t *out, int use_cache);
int hydro_batch_set_profiling(hydro_batch_t *b, int enable);
int hydro_batch_get_profile(hydro_batch_t *b, double ms[HYDRO_NPHASES],
                            long long launches[HYDRO_NPHASES], int reset);
int hydro_batch_set_mlp(hydro_batch_t *b, const void *mlp);
int hydro_batch_set_logger(hydro_batch_t *b, float *records, long long capacity,
                           unsigned long long seed, double rate_smooth, double rate_strong);
long long hydro_batch_logger_count(hydro_batch_t *b);

/* ------------------------------------------------------------------------
 * Measurement: the bandwidth a plain streaming kernel reaches on this GPU,
 * the practical ceiling beside the published HBM peak for the sweeps, which
 * read and write their state once per sweep (measured in bench.py).
 * ------------------------------------------------------------------------ */
/* Copy nbytes from src to dst (device memory owned by the caller, both
 * 16-byte aligned, not overlapping), asynchronously on hip_stream: one 8 KiB
 * chunk per block, 4-byte nontemporal loads and stores.  nbytes must be
 * a multiple of 16 (0 is a no-op).  HYDRO_EINVAL for a NULL pointer, a
 * misaligned pointer or size, or overlapping ranges; HYDRO_EDEVICE if the
 * launch fails. */
int hydro_stream_copy(void *dst, const void *src, long long nbytes, void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* HYDRO_H */
