/*
 * gpweno.h -- C ABI of libgpweno: the GP-WENO finite-difference (FD-Prim)
 * scheme for the compressible Euler equations on static uniform grids (periodic,
 * outflow or reflecting boundaries per axis side), on one AMD Instinct MI355X
 * (gfx950).
 *
 * Method (Reyes, Lee, Graziani, Tzeferacos, "A variable high-order
 * shock-capturing finite difference method with GP-WENO"):
 *   - point values of the conserved variables U = (rho, rho u[, rho v[, rho w]], E)
 *     (Sec. 2, Eq. (euler)) are advanced by the conservative difference of
 *     numerical fluxes, Eq. (disc_fd);
 *   - Riemann states at the faces x_{i+-1/2} are interpolated per direction by
 *     GP-WENO on characteristic variables (Sec. 3.2-3.3, Sec. 4 step 2, Sec. 7);
 *   - face fluxes come from an HLLC Riemann solver (Eq. (riemann_prob)) and are
 *     corrected to high order with alpha = -1/24, beta = 3/640
 *     (Eqs. (numFlux_cor), (FD-ders)), optionally with the next term of the
 *     same series (gpweno_options.flux_corr_terms);
 *   - time integration is third-order SSP (TVD) Runge-Kutta.
 *
 * Conventions shared by every entry point
 *   - Status: every function returns an int, GPWENO_OK (0) on success or a
 *     negative gpweno_status. Nothing is printed, nothing exits; the text of the
 *     last failure is available from gpweno_last_error().
 *   - Units: ell and sigma are physical lengths (pass 12*dx and 3*dx for the
 *     paper's usual ell/dx = 12, sigma/dx = 3, Sec. 3.4). gamma is the ratio of
 *     specific heats (not the paper's linear weights).
 *   - State layout: float64, structure of arrays [nv][nz][ny][nx], x fastest,
 *     nv = 2 + ndim, conserved variables in the order (rho, rho u, rho v, rho w, E)
 *     restricted to the grid's dimension. Values are point values at cell centres
 *     x_i = lo + (i + 1/2) dx.
 *   - Ownership: the caller allocates and owns the device state and the device
 *     workspace (any allocator, e.g. PyTorch); the library never frees them.
 *     A context owns only its small control block and host-side tables.
 *   - Streams: work is enqueued on the context's stream (gpweno_options.stream,
 *     a hipStream_t; NULL means the default stream). Calls documented as
 *     blocking synchronise that stream; the others return after enqueueing.
 *   - Threads: a context is used by one host thread at a time.
 */
#ifndef GPWENO_H
#define GPWENO_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GPWENO_OK = 0,
    GPWENO_EINVAL = -1,    /* invalid argument */
    GPWENO_ENOMEM = -2,    /* allocation failed */
    GPWENO_EHIP = -3,      /* a HIP runtime call failed */
    GPWENO_ENONPHYS = -4,  /* a non-physical state (rho <= 0, p <= 0 or NaN) was produced */
    GPWENO_ESTATE = -5     /* call not valid in the context's current state (e.g. not bound) */
} gpweno_status;

typedef enum {
    GPWENO_FP64 = 0,       /* all arithmetic in float64 */
    GPWENO_FP32 = 1        /* sweep arithmetic in float32; state, flux differences,
                              RK combination, dt and conservation sums in float64 */
} gpweno_precision;

/* Boundary kind of one side of an axis. */
typedef enum {
    GPWENO_BC_PERIODIC = 0, /* periodic images (both sides of the axis) */
    GPWENO_BC_OUTFLOW = 1,  /* zero-gradient ghosts: copies of the boundary cell */
    GPWENO_BC_REFLECT = 2   /* reflecting wall: mirror image about the boundary face,
                               normal velocity reversed; needs n >= R + 3 (R + 4
                               with flux_corr_terms = 3) */
} gpweno_bc;

/* Uniform grid. Axes beyond ndim are ignored. */
typedef struct {
    int ndim;              /* 1, 2 or 3 */
    int n[3];              /* cells per axis */
    double lo[3];          /* domain lower corner */
    double hi[3];          /* domain upper corner */
    int bc[3][2];          /* gpweno_bc per axis, [axis][0 = low side, 1 = high side];
                              all zero = periodic everywhere. A periodic axis must be
                              periodic on both sides. The paper's shock problems use
                              outflow boundaries (Sec. 7). */
} gpweno_grid;

/* Interpolation scheme of the Riemann states. GP-WENO is the paper's method;
 * the other two are its comparison schemes (Sec. 6.2, Table (weno-vortex)):
 * polynomial WENO interpolation (Lagrange weights on the sub-stencils, their
 * linear weights) with the classical Jiang-Shu smoothness indicators, or with
 * the GP smoothness indicators of Eq. (beta-eigen). All three use the
 * nonlinear weights of Eq. (weights) with p = 2, eps = 1e-36. */
typedef enum {
    GPWENO_GP_WENO = 0,    /* GP weights, GP linear weights, GP indicators (R = 1..3) */
    GPWENO_WENO_JS = 1,    /* polynomial weights, Jiang-Shu indicators (R = 1, 2) */
    GPWENO_WENO_GP = 2,    /* polynomial weights, GP indicators with sigma (R = 1..3) */
    GPWENO_GP_AO = 3       /* adaptive-order GP of App. A: R = 3 is GP-AO(3,2,3), R = 2 is
                              GP-AO(2,3). GP-CWENO on the 3-point sub-stencils (linear
                              weights of Eq. (CWENO-lin), gamma_HI = gamma_LO = 0.85)
                              hybridised with the 5- and 7-point GP interpolations
                              (Eqs. (nonlin-AO), (GP-AO), (AO-recursive)); indicators
                              are the full negative log-likelihood of Eq. (log-like)
                              with K_N(sigma). The paper uses sigma/dx = 1.8 with it. */
} gpweno_scheme;

typedef struct {
    int precision;         /* gpweno_precision */
    double cfl;            /* CFL number of the time-step rule (default 0.4) */
    double fixed_dt;       /* > 0: use this time step instead of the CFL rule */
    int positivity_fallback; /* 1: a Riemann state with rho <= 0 or p <= 0 is replaced
                                by the cell-centre state (default 0) */
    void *stream;          /* hipStream_t, NULL = default stream */
    int nonzero_mean;      /* 1: the GP smoothness indicators (GP-WENO, WENO-GP) see
                              the sub-stencil data minus the centre cell's value,
                              the non-zero-mean variant of Sec. 7 (scalar advection);
                              0: zero mean, the paper's default (default 0). No
                              effect on the Jiang-Shu indicators, which ignore
                              constants. */
    int flux_corr_terms;   /* terms of the high-order flux correction of Eq.
                              (numFlux_cor): 2 (default, the paper's): alpha = -1/24
                              on the second and beta = 3/640 on the fourth difference
                              of the face fluxes; 3: also -5/7168 on the sixth
                              difference, the next term of the same series (the
                              "+ ..." of that equation), exact for face fluxes that
                              are polynomials of degree <= 7 instead of 5. 3 needs
                              one more ghost cell per side (R + 4) and is offered for
                              the schemes with GP indicators of zero mean (GP-WENO,
                              WENO-GP); EINVAL otherwise. */
} gpweno_options;

typedef struct gpweno_ctx gpweno_ctx;

/* Pre-simulation step (Sec. 4 step 1): builds the GP weights w_m at x_{i+-1/2}
 * (Eqs. (kmat), (kstar), (q-intrp)), the linear weights gamma_m as the
 * least-squares solution of Eq. (gamm-system) with M of Eq. (M-mat), and the
 * eigen-projections P_i = v_i / sqrt(lambda_i) of K_m(sigma) (Eq. (beta-eigen)),
 * in binary128 and rounded to float64, for every direction.
 * grid: host pointer, copied. R: stencil radius, 1..3. ell, sigma: physical
 * length scales, sigma > dx on every axis (Sec. 3.4: sigma <= dx is unstable).
 * gamma: ratio of specific heats, > 1. Every axis needs n >= 2. On success *out
 * receives a context with default options; the device in use is the current
 * HIP device. Errors: EINVAL for invalid arguments, ENOMEM/EHIP on allocation.
 * Host-side work plus a control block from a per-device pool (allocated 64 at
 * a time, reused after gpweno_destroy). */
int gpweno_init(const gpweno_grid *grid, int R, double ell, double sigma, double gamma,
                gpweno_ctx **out);

/* gpweno_init for any gpweno_scheme: the same context, with the scheme's tables
 * in place of the GP ones. ell is used only by GPWENO_GP_WENO; sigma (> dx) by
 * the two schemes with GP indicators, and validated for all. Errors: as
 * gpweno_init, and EINVAL for an unknown scheme or WENO-JS with R = 3. */
int gpweno_init_scheme(const gpweno_grid *grid, int scheme, int R, double ell, double sigma,
                       double gamma, gpweno_ctx **out);

/* Options (host pointer, copied). Changing the precision, the positivity
 * flag, the non-zero-mean flag, the correction terms or the stream drops any
 * captured graph; a context with a bound state or captured graphs first waits
 * for its current stream (blocking: graph launches may still be in flight
 * there, and work on a new stream comes after them). Errors: EINVAL, EHIP. */
int gpweno_set_options(gpweno_ctx *ctx, const gpweno_options *opt);
int gpweno_get_options(const gpweno_ctx *ctx, gpweno_options *opt);

/* Number of float64 values in the state: nv * ncells. */
size_t gpweno_state_count(const gpweno_ctx *ctx);

/* Bytes of device workspace gpweno_bind needs (two RK stage states, the
 * direction accumulator and reduction partials), 256-byte aligned. */
size_t gpweno_workspace_bytes(const gpweno_ctx *ctx);

/* Binds the caller's device state (float64, layout above, gpweno_state_count
 * values) and workspace (gpweno_workspace_bytes bytes, 256-byte aligned). Both
 * stay owned by the caller and must outlive the binding. Resets t and the step
 * count to 0, and enqueues the CFL speed reduction of the current state (so the
 * state must hold valid data before the first step; call gpweno_set_time after
 * changing it). Rebinding a context whose captured graphs may still run waits
 * for its stream first and drops them. Errors: EINVAL for NULL or misaligned
 * pointers, EHIP. */
int gpweno_bind(gpweno_ctx *ctx, double *d_state, void *d_workspace);

/* Sets the simulation time and step count, and recomputes the CFL speed of the
 * bound state (enqueued). Use after the caller rewrote the state. ESTATE if
 * not bound. */
int gpweno_set_time(gpweno_ctx *ctx, double t, long nsteps);

/* One SSP-RK3 step: dt = cfl / max_i sum_d (|u_d|+c)/dx_d from the state at the
 * start of the step (or fixed_dt), clipped so that t does not pass t_final;
 * no-op when t >= t_final. The state is updated in place.
 * dt_out: NULL enqueues the step and returns at once (asynchronous); failures
 * inside the step are then reported by the next blocking call (gpweno_get_time /
 * gpweno_run) as ENONPHYS. Non-NULL (host pointer) waits for the step and
 * stores the dt it took (0 if it did not run: t >= t_final or an earlier
 * failure), returning ENONPHYS if the step produced a non-physical state.
 * ESTATE if not bound. */
int gpweno_step(gpweno_ctx *ctx, double t_final, double *dt_out);

/* The k-th of the 3 * ndim kernel launches that make up one gpweno_step
 * (stage k / ndim + 1, direction k % ndim), enqueued on its own. Enqueuing
 * k = 0 .. 3 ndim - 1 in order performs exactly one step, with the end time and
 * step limit left as the last gpweno_step / gpweno_run set them. For
 * instrumentation (e.g. timing each kernel with events on the context's stream).
 * Errors: EINVAL for k out of range, ESTATE if not bound. */
int gpweno_step_kernel(gpweno_ctx *ctx, int k);

/* Advances until t >= t_final or max_steps more steps were taken (max_steps < 0:
 * no limit). Blocking. Steps are replayed from captured HIP graphs. On return
 * *nsteps_out (nullable) holds the steps taken by this call and *t_out (nullable)
 * the time reached. Returns ENONPHYS if a stage produced rho <= 0, p <= 0 or a
 * NaN; the remaining launches of that step are skipped and no further step
 * starts, so the state then holds either the state at the start of the
 * failing step (failure in stage 1 or 2) or that step's non-physical output
 * (stage 3). gpweno_set_time clears the condition. */
int gpweno_run(gpweno_ctx *ctx, double t_final, long max_steps, long *nsteps_out, double *t_out);

/* Blocking: current time, the last step's dt, and the total step count
 * (each nullable). Returns ENONPHYS if a non-physical state was detected, with
 * the smallest flagged cell index in the error text and in *bad_cell of
 * gpweno_get_failure. */
int gpweno_get_time(gpweno_ctx *ctx, double *t, double *dt, long *nsteps);

/* Blocking: whether a non-physical state was detected (*failed = 1) and the
 * smallest flagged cell index (*bad_cell, -1 if none); each nullable. */
int gpweno_get_failure(gpweno_ctx *ctx, int *failed, long *bad_cell);

/* One evaluation of the right-hand side of Eq. (disc_fd) for an arbitrary device
 * state d_U (same layout as the bound state), written to d_L (same size):
 * L = -sum_d (fhat_{i+1/2} - fhat_{i-1/2}) / dx_d. Enqueued. Needs no bound
 * state or workspace; d_U and d_L must not overlap. Errors: EINVAL. */
int gpweno_rhs(gpweno_ctx *ctx, const double *d_U, double *d_L);

/* One direction's term of the right-hand side of Eq. (disc_fd):
 * -(fhat_{i+1/2} - fhat_{i-1/2}) / dx_dir for every cell, from the device state
 * d_U, written to d_L (accumulate = 0) or added to d_L (accumulate = 1). This is
 * exactly one launch of the direction's sweep kernel. dir < ndim. Enqueued.
 * d_U and d_L must not overlap. Errors: EINVAL. */
int gpweno_rhs_dir(gpweno_ctx *ctx, int dir, const double *d_U, double *d_L, int accumulate);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): gpweno_step (dt_out
 * NULL, enqueued) for a state the caller passes, d_state (device pointer, the
 * layout of gpweno_bind, updated in place), with the two RK stage states and
 * the direction accumulator in a scratch area the library holds in device
 * memory instead of a bound workspace. It allocates nothing (no hipMalloc,
 * hipFree or allocating library call). The CFL time step comes from d_state
 * (its speed is reduced first, into the context's control block), and the
 * context's time and step count advance as with gpweno_step; its bound state
 * and workspace, if any, are not touched. The scratch is 64 MiB per device
 * (GPWENO_NOALLOC_SCRATCH_BYTES): 2 + (ndim > 1) arrays of nv * ncells float64,
 * each rounded up to 256 bytes, must fit, e.g. 2D grids up to about 699,000
 * cells, 3D up to about 559,000; a larger grid returns EINVAL. Every call on a
 * device shares that device's one scratch area and keeps the last call's
 * contents (no part needs to start at zero): calls that overlap on one device
 * (other streams, other threads) race. The context must have been created on
 * the device the call runs on. Errors: EINVAL (NULL or misaligned state,
 * grid too large), EHIP (the scratch address could not be taken at
 * gpweno_init). */
#define GPWENO_NOALLOC_SCRATCH_BYTES (64u << 20)
int gpweno_step_noalloc(gpweno_ctx *ctx, double *d_state, double t_final);

/* Blocking: float64 sums over all cells of each conserved field of the bound
 * state, written to host out[nv], by a deterministic device reduction. */
int gpweno_conserved_sums(gpweno_ctx *ctx, double *out);

/* Host-only, no device work: the pre-simulation tables this context uses along
 * axis dir (0 <= dir < ndim), built by gpweno_init from ell/dx_dir and
 * sigma/dx_dir (Sec. 4 step 1), as float64 host arrays (each nullable, caller
 * owned), row-major:
 *   w_sub[2][R+1][R+1]: GP (or polynomial) weights w_m of sub-stencil m = 0..R
 *     (nodes m-R .. m relative to the centre cell) at x_* = +1/2 ([0]) and
 *     -1/2 ([1]), Eq. (q-intrp) on K_m of Eq. (kmat);
 *   gam[2][R+1]: linear weights gamma_m at x_* = +1/2 and -1/2, the least-squares
 *     solution of Eq. (gamm-system);
 *   P[R+1][R+1]: rows v_i / sqrt(lambda_i) of K_m(sigma), Eq. (beta-eigen), so
 *     that beta_m = sum_i (P_i . f_m)^2 for every m. The Jiang-Shu indicators of
 *     GPWENO_WENO_JS differ per sub-stencil (gpweno_compute_tables gives them):
 *     P must be NULL there.
 * For GPWENO_GP_AO, w_sub, gam and P are those of its 3-point sub-stencils
 * (R + 1 reads 3 in the sizes; gamma: the CWENO linear weights; the 5- and
 * 7-point tables come from gpweno_compute_ao_tables). The float32 path uses these values
 * rounded to float32. Errors: EINVAL (NULL context, dir out of range, P for
 * WENO-JS). */
int gpweno_get_tables(const gpweno_ctx *ctx, int dir, double *w_sub, double *gam, double *P);

/* Host-only: accuracy of this context's tables, the largest relative difference
 * over all axes between the weights solved directly at x_* = -1/2 and the
 * mirror image of those at x_* = +1/2, which agree exactly in exact arithmetic.
 * K of Eq. (kmat) loses conditioning as ell/dx grows (R = 3 in binary128:
 * 1e-16 at 40 dx, 2e-14 at 51 dx, 2e-13 at 60 dx, 1e-12 at 80 dx, 7e-8 at
 * 192 dx; R <= 2 stays below 1e-15 up to 220 dx), and the linear weights are
 * only as accurate as this residual (within a factor of about 5 against
 * 60-digit solves). A context whose residual exceeds 1e-13 runs in
 * GPWENO_FP32 only: gpweno_set_options refuses GPWENO_FP64 for it, and it
 * starts in GPWENO_FP32. Errors: EINVAL. */
int gpweno_table_residual(const gpweno_ctx *ctx, double *residual);

/* Test hook (enqueued on the context's stream): overwrites the bound state's
 * density and total energy at cell index `cell` (0 <= cell < ncells, x fastest)
 * with -1, a non-physical state. The next stage that reads it produces
 * non-finite or non-physical values in the cells whose stencils contain it; the
 * physical check of the stage flags the step, which then reports ENONPHYS
 * through the normal path (gpweno_run, gpweno_get_time, gpweno_batch_status),
 * with the smallest flagged cell index, which lies within R + 3 cells (R + 4
 * with flux_corr_terms = 3) of `cell` along each axis. No GPU fault is
 * involved. Errors: EINVAL (cell out of range), ESTATE (not bound). */
int gpweno_debug_poison(gpweno_ctx *ctx, long cell);

/* Host-only (no device needed): the pre-simulation tables of gpweno_init_scheme
 * for a scheme (gpweno_scheme), stencil radius R and length scales in units of
 * dx (ell_over_dx, sigma_over_dx; ell is unused by the polynomial schemes).
 * Outputs are host arrays, row-major, padded to 4: w_plus[4][4], w_minus[4][4]
 * (sub-stencil m = 0..R, node j = 0..R; sub-stencil m holds nodes m-R..m
 * relative to the centre cell), gam_plus[4], gam_minus[4], and P[4][4][4] with
 * beta_m = sum_i (P[m][i] . f_m)^2 (GP: row i is v_i / sqrt(lambda_i) of
 * K_m(sigma), Eq. (beta-eigen), the same for every m). Any output may be NULL.
 * Errors: EINVAL (also WENO-JS with R = 3). */
int gpweno_compute_tables(int scheme, int R, double ell_over_dx, double sigma_over_dx,
                          double *w_plus, double *w_minus, double *gam_plus,
                          double *gam_minus, double *P);

/* Host-only: the mirror residual (see gpweno_table_residual) of the tables
 * gpweno_compute_tables builds for the same arguments, into *residual.
 * Errors: EINVAL. */
int gpweno_compute_table_residual(int scheme, int R, double ell_over_dx, double sigma_over_dx, double *residual);

/* Host-only: the extra tables of GPWENO_GP_AO for length scales in units of dx.
 * w7[2][7] and w5[2][5]: GP weights of the 7- and 5-point stencils (nodes -3..3,
 * -2..2) at x_* = +1/2 (row 0) and -1/2 (row 1), Eq. (q-intrp); P7[7][7],
 * P5[5][5], P3[3][3]: rows v_i / sqrt(lambda_i) of K_N(sigma); c[3]: for N = 7,
 * 5, 3, N/2 log(2 pi) + 1/2 log det K_N(sigma) (Eq. (log-like)). Any output may
 * be NULL. Errors: EINVAL. */
int gpweno_compute_ao_tables(double ell_over_dx, double sigma_over_dx, double *w7, double *w5,
                             double *P7, double *P5, double *P3, double *c);

/* Sets the end time and the absolute step limit (step_limit < 0: none) of the
 * context's runs without stepping (enqueued). gpweno_batch_run honours them;
 * gpweno_step and gpweno_run set their own. ESTATE if not bound. */
int gpweno_set_end(gpweno_ctx *ctx, double t_final, long step_limit);

/* ---- Batched execution of many independent problems ------------------------
 * A batch advances a set of bound contexts together: every launch of the step
 * sequence covers all problems of a group (one kind: same ndim, R, precision,
 * scheme and indicator kind, flux-correction terms, boundary kinds per axis and
 * per-axis tables) with one kernel whose blocks are dealt problem by problem. Each
 * problem keeps its own dt, time, end time and step limit in its own control
 * block; a problem that is done skips its blocks. A block computes exactly
 * what the single-problem sweep computes for its cells, so each problem's
 * result does not depend on the rest of the batch.
 * Serves a request loop (continuous batching): the caller changes the set as
 * problems arrive and finish (gpweno_batch_set), advances it in chunks of
 * steps (gpweno_batch_run) and polls progress (gpweno_batch_status).
 * All calls on a batch, and the contexts' own work, must be ordered on one
 * stream (pass the contexts' stream). */
typedef struct gpweno_batch gpweno_batch;

/* Creates an empty batch on the current device. Errors: ENOMEM, EHIP. */
int gpweno_batch_create(gpweno_batch **out);

/* Sets the batch's problems: n (<= 4096) distinct bound contexts on the batch's
 * device, of at most 64 kinds. Enqueued: the batch's device work tables (the
 * problems' descriptors and block owners) are written by stream-ordered copies
 * from a pinned staging ring, so launches enqueued before the call still see
 * the old set and later ones the new; the host does not wait for the stream
 * (except when the tables outgrow their capacity, which doubles, or when the
 * previous call used another stream). The captured step graph reads the
 * tables through fixed addresses and keeps serving the new set while its kinds
 * of problems stay the same. The contexts must stay alive and bound until they
 * are removed by a later gpweno_batch_set and that set's launches have begun
 * (destroying a context synchronises its stream). n = 0 empties the batch.
 * Errors: EINVAL (NULL, repeated or unbound context, mixed devices, too many
 * kinds), ENOMEM, EHIP. */
int gpweno_batch_set(gpweno_batch *b, gpweno_ctx *const *ctxs, int n, void *stream);

/* Enqueues nsteps batched steps (nsteps >= 1) on stream by replaying captured
 * graphs of eight batched steps and of one (nsteps / 8 and nsteps % 8 times),
 * per kind of problem (captured on first use, and again only when the kinds of
 * problems in the set change). With several kinds, each kind's graphs are
 * replayed on a stream of the batch's own that waits for stream first and that
 * stream then waits for, so kinds (which share no data) may run side by side
 * while everything stays ordered on stream. Every launch has one block per logical block of its group; after
 * a set change of the same kinds the grids of the captured launches are
 * updated in place on the instantiated graphs before the next replay.
 * Errors: EINVAL, EHIP. */
int gpweno_batch_run(gpweno_batch *b, int nsteps, void *stream);

/* Blocking: for every problem of the set, in set order, its time, last dt, step
 * count and error flag (1: non-physical state) into host arrays of length n
 * (each nullable), read on stream after the steps enqueued so far (on another
 * stream than the last set or run, that stream is waited for first).
 * Errors: EINVAL, EHIP. */
int gpweno_batch_status(gpweno_batch *b, double *t, double *dt, long *nsteps, int *err, void *stream);

/* Number of times the batch has captured its step graphs (all kinds' graphs at
 * once count as one capture; instrumentation; -1 for NULL). A set change that keeps the kinds of problems (dimension, R,
 * precision, scheme, boundary kinds, flux correction, tables) in the same order
 * does not add one, whatever the problems' sizes: the captured launches read
 * the set through the work tables, and their grids are updated in place. */
long gpweno_batch_captures(const gpweno_batch *b);

/* Waits for the stream of the batch's last set or run (the default stream
 * too, when that was the one) and for its per-kind streams, and frees its
 * resources. NULL is ignored. */
void gpweno_batch_destroy(gpweno_batch *b);

/* Text of the last failure on this batch (NULL: the thread's last failure of
 * a call given a NULL batch). Never NULL. */
const char *gpweno_batch_last_error(const gpweno_batch *b);

/* Text of the last failure on this context (ctx may be NULL for failures of
 * gpweno_init and of calls given a NULL context). Never NULL. */
const char *gpweno_last_error(const gpweno_ctx *ctx);

/* Releases the context's own resources (not the caller's buffers). Synchronises
 * the context's stream first (NULL: the default stream). NULL is ignored. */
void gpweno_destroy(gpweno_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* GPWENO_H */
