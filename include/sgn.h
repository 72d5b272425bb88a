/*
 * sgn.h -- C ABI of the MI355X (gfx950) solver for the energy-conserving
 * split-form SBP semi-discretization of the two-dimensional hyperbolized
 * Serre-Green-Naghdi equations with variable bathymetry (arXiv 2601.02540).
 *
 * Problem statement followed by the calls (paper references):
 *   unknowns h, u, v, w, eta and static bathymetry b, gravity g, relaxation
 *   parameter lambda: eq. (2D_hyperbolic_SGN), Section 3.2;
 *   nodal grid and SBP operators (D, M): Section 2.2 and Remark "Concrete SBP
 *   operators and SATs" (second-order central differences; periodic, or
 *   first-order one-sided closures with a trapezoid mass matrix);
 *   right-hand side: eq. (sd_periodic_2D_SGN) (periodic) and eq. (semi_2D)
 *   (reflecting walls, weak SATs in the h equation only);
 *   total mass 1^T M h and energy 1^T M E: Theorems 1 and 2;
 *   auxiliary initialization: eq. (initialization), Section 6.
 *
 * Memory layout.  A state q is five contiguous planes [h, u, v, w, eta], each
 * ny*nx values, row-major with x (index i) fastest: q[f*nx*ny + j*nx + i].
 * The bathymetry is one such plane.  All array arguments are DEVICE pointers
 * on the context's device, in the context's storage type (double for
 * SGN_F64, float for SGN_F32), unless documented otherwise.  Scalars returned
 * to the caller (mass, energy, rates, dt) are host doubles.
 *
 * Node placement: a periodic axis [lo, hi) has N nodes spaced (hi-lo)/N (the
 * right end point is the image of the left one); a reflecting axis [lo, hi]
 * has N nodes spaced (hi-lo)/(N-1) including both walls.
 *
 * Ownership.  The caller owns every array it passes.  The context owns a copy
 * of b, the Runge-Kutta scratch planes, reduction partials, captured graphs
 * and a device health flag.  Nothing is retained past a call except the copy
 * of b and the stream.
 *
 * Asynchrony.  Calls that return no host value (set_bathymetry, init_aux, rhs,
 * step) only enqueue work on the context's stream and return.  Calls that
 * return host values (mass, energy, mass_energy, rates, cfl_dt, check)
 * synchronize the stream.  Launch failures are reported immediately.
 *
 * Errors.  Every call returns an sgn_status; no exception crosses the ABI.
 * A call that fails leaves a message for sgn_last_error().  Kernels raise a
 * device flag when a step produces h <= 0 or a non-finite value (the method
 * has no wetting and drying); the flag is reported as SGN_E_NONPOS_DEPTH or
 * SGN_E_NONFINITE by the next synchronizing call and then cleared.
 *
 * Threading.  One context belongs to one stream; calls on the same context
 * must not overlap.  Different contexts are independent.
 */
#ifndef SGN_H
#define SGN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SGN_OK = 0,
  SGN_E_ARG = -1,           /* null pointer, non-finite or negative parameter */
  SGN_E_SHAPE = -2,         /* fewer than 4 nodes on an axis, empty domain, overflow */
  SGN_E_UNSUPPORTED = -3,   /* option not available for this dtype/boundary combination */
  SGN_E_HIP = -4,           /* HIP runtime error (message has the HIP error string) */
  SGN_E_NONPOS_DEPTH = -5,  /* a kernel saw h <= 0 */
  SGN_E_NONFINITE = -6,     /* a kernel saw NaN or Inf in the state */
  SGN_E_ALLOC = -7,         /* device allocation failed */
  SGN_E_STATE = -8          /* call out of order (e.g. bathymetry never set) */
} sgn_status;

typedef enum { SGN_PERIODIC = 0, SGN_REFLECTING = 1 } sgn_bc;
typedef enum { SGN_F64 = 0, SGN_F32 = 1 } sgn_dtype;

/* Source terms added to the right-hand side at stage time.
 * SGN_SRC_MMS: the manufactured solution of Section 6.1.2 (domain [-1,1]^2):
 * the analytic residual of eq. (2D_hyperbolic_SGN) in the evolved
 * (primitive) variables is added to every stage, evaluated at t_n + c_s dt. */
typedef enum { SGN_SRC_NONE = 0, SGN_SRC_MMS = 1 } sgn_source;

typedef struct {
  int32_t nx, ny;           /* nodes per axis, each >= 4 */
  double xmin, xmax;        /* domain along x (xmax > xmin) */
  double ymin, ymax;        /* domain along y (ymax > ymin) */
  int32_t bc_x, bc_y;       /* sgn_bc per axis (the two may differ) */
  double g;                 /* gravitational acceleration, > 0 */
  double lambda;            /* hyperbolization (relaxation) parameter, >= 0 */
  int32_t dtype;            /* sgn_dtype: storage and arithmetic of the state */
  int32_t source;           /* sgn_source */
} sgn_params;

typedef struct sgn_ctx sgn_ctx;

/* Options (sgn_set_option).
 * SGN_OPT_STEP_PATH: how sgn_step evaluates one RK4 step.
 *   SGN_PATH_FUSED (default): one kernel per step; the three intermediate
 *     stages stay in LDS (a four-node halo, evaluated redundantly in rings
 *     around each tile).  11 values of HBM traffic per node and step.
 *   SGN_PATH_PAIRS: two kernels, each fusing two stages; the intermediate
 *     stage stays in LDS.  37 values per node and step.
 *   SGN_PATH_STAGES: four kernels, one per stage.  84 values per node and step.
 *   On the fused and pair paths the state alternates between the caller's
 *   buffer and a context buffer, so steps go in twos; an odd final step runs on
 *   the four-stage path.
 * SGN_OPT_TILE_Y: 8, 16 or 24.  Tile height of the stage and pair kernels (64
 *   wide; default 8 for SGN_F64, 16 for SGN_F32) and of the step kernel's tile
 *   (8 selects 64 x 8, 16 selects 32 x 16, 24 selects 32 x 24: three owned
 *   nodes per thread and the fewest redundant ring evaluations; default 24
 *   when the grid holds at least 1024 tiles of 32 x 24, 16 otherwise).
 *   8 and 16 set both; 24 sets the step tile and height 16 for the stage and
 *   pair kernels.  With a 32 x 24 step tile, steps that save stage states or
 *   add source terms, and the adaptive pair's attempt kernel on grids with a
 *   wall, run 32 x 16 tiles.  Every tile shape forms the same values.
 * SGN_OPT_ADJOINT_STORE: bytes of device memory (>= 0; default 0) that
 *   sgn_gauge_loss_grad may fill with the states and stage states of the last
 *   steps of its forward rollout, so that its reverse sweep need not recompute
 *   them (see there). */
typedef enum { SGN_OPT_STEP_PATH = 0, SGN_OPT_TILE_Y = 1, SGN_OPT_ADJOINT_STORE = 2 } sgn_option;
typedef enum { SGN_PATH_PAIRS = 0, SGN_PATH_STAGES = 1, SGN_PATH_FUSED = 2 } sgn_step_path;

/* Create a context on the current HIP device.  stream is a hipStream_t (NULL
 * for the null stream).  Allocates the Runge-Kutta scratch (three states), a
 * bathymetry plane and the reduction partials.  On failure *out is NULL. */
sgn_status sgn_create(const sgn_params* params, void* stream, sgn_ctx** out);

/* Free everything the context owns (synchronizes its stream first). NULL is a no-op. */
sgn_status sgn_destroy(sgn_ctx* ctx);

/* Change the stream later calls are enqueued on (invalidates captured graphs). */
sgn_status sgn_set_stream(sgn_ctx* ctx, void* stream);

/* Set an sgn_option (drops captured graphs).  SGN_E_ARG / SGN_E_UNSUPPORTED on
 * unknown options or values. */
sgn_status sgn_set_option(sgn_ctx* ctx, int32_t option, int64_t value);

/* Copy the bathymetry b (device, one plane) into the context.  Required before
 * any call that evaluates the right-hand side or the energy. */
sgn_status sgn_set_bathymetry(sgn_ctx* ctx, const void* b);

/* In place on q: eta = h and w = -h (D_x u + D_y v) + 3/2 (u D_x b + v D_y b)
 * with the discrete operators (eq. (initialization)).  h, u, v are read. */
sgn_status sgn_init_aux(sgn_ctx* ctx, void* q);

/* dq = right-hand side of the semi-discretization at state q and time t (t
 * only matters with a source).  q and dq must not overlap. */
sgn_status sgn_rhs(sgn_ctx* ctx, const void* q, void* dq, double t);

/* Advance q in place by nsteps steps of the classical four-stage Runge-Kutta
 * method with fixed step dt, starting at time t0, on the context's step path
 * (SGN_OPT_STEP_PATH).  nsteps == 0 is a no-op.  Without a source the steps
 * are replayed from a captured HIP graph. */
sgn_status sgn_step(sgn_ctx* ctx, void* q, double dt, int64_t nsteps, double t0);

/* Capture and instantiate the HIP graphs that sgn_step(ctx, q, dt, nsteps, .)
 * replays (one for 8-step runs, one for the 1- or 2-step remainder), so that a
 * later sgn_step with the same q, dt and path pays no capture; enqueues no
 * work and leaves q untouched.  Same argument rules as sgn_step; a no-op with
 * a source term (those steps are launched directly) or nsteps == 0.  Graphs are
 * dropped by sgn_set_option, sgn_set_stream and sgn_set_bathymetry. */
sgn_status sgn_prepare_step(sgn_ctx* ctx, void* q, double dt, int64_t nsteps);

/* Relaxation RK4 (fully discrete energy conservation; the extension the paper
 * names in its conclusions).  Each step takes the classical RK4 update
 * d = q_RK4 - q_n (computed on the context's step path into the context's
 * scratch state) and sets q_{n+1} = q_n + gam_n d, t_{n+1} = t_n + gam_n dt, with
 * gam_n the root near 1 of E(q_n + gam d) = E(q_n), E the total energy of
 * Theorem 2.  Since the semi-discretization conserves E, the fully discrete E
 * is then conserved to rounding and the method keeps fourth order in time.
 * gam_n comes from two Newton iterations from 1 on the device (FP64 reductions,
 * no host synchronization per step; steps are replayed from a captured graph);
 * a step without a root in [1/2, 3/2] keeps gam = 1.  The state stays in q.
 * If t_end is not NULL it receives t0 + sum_n gam_n dt (synchronizes, and
 * reports the health flag); otherwise the call is asynchronous.  Requires no
 * source term (SGN_E_UNSUPPORTED). */
sgn_status sgn_step_relaxation(sgn_ctx* ctx, void* q, double dt, int64_t nsteps, double t0, double* t_end);

/* Classical RK4 like sgn_step, recording the totals of every step: after
 * step k (1-based), series[2 (k-1)] = mass and series[2 (k-1) + 1] = energy of
 * the state (the definitions of sgn_mass_energy).  The steps run on the step
 * kernel whatever the step path (every path forms the same states), which
 * reduces the totals of each tile from the values it writes, so the series
 * costs no pass over the state (totals summed in FP64, compensated,
 * deterministic; they agree with sgn_mass_energy to rounding).  series: device
 * memory, 2 nsteps doubles, FP64 whatever the dtype; not NULL unless nsteps is
 * 0 (a no-op).  nsteps < 2^30 (SGN_E_ARG otherwise).  Steps are
 * replayed from a captured graph; asynchronous.  Requires no source term
 * (SGN_E_UNSUPPORTED). */
sgn_status sgn_step_totals(sgn_ctx* ctx, void* q, double dt, int64_t nsteps, double* series);

/* Result of sgn_step_adaptive (host struct filled by the call). */
typedef struct {
  double t;             /* time reached: t_end unless the attempt limit stopped the run */
  double h_next;        /* the step the controller proposes next */
  double last_err;      /* error norm of the last attempt */
  int64_t attempts;     /* accepted + rejected */
  int64_t accepted;
  int64_t rejected;
  int32_t reached_end;  /* 1 when t == t_end */
} sgn_adaptive_result;

/* Adaptive time integration with the kind of method the paper uses (Section
 * "Numerical Experiments": an explicit third-order, five-stage Runge-Kutta
 * method with the first-same-as-last property and an embedded error estimate
 * driving the step; the paper runs it at rtol = atol = 1e-6).  The paper cites
 * the method without its coefficients; this pair has that shape:
 *   Y_{i+1} = y_n + h c_{i+1} k_i, c = (0, 1/3, 3/4, 4/5, 3071/3720),
 *   y_{n+1} = y_n + h sum b_i k_i, b = (7200668/46553289, 1701/5053,
 *   6098/15159, 350/5053, 18600/500573): order 3, stability polynomial
 *   1 + z + z^2/2 + z^3/6 + z^4/31 + z^5/163;
 *   error estimate e = h b_5 (k_5 - (1 - c_5) k_1 - c_5 k_6), k_6 = f(y_{n+1})
 *   the next step's k_1 (an embedded second-order method);
 *   err = RMS over all 5N values of e / (atol + rtol max(|y_n|, |y_{n+1}|)),
 *   accepted when err <= 1; PI control h_new = h 0.9 err^(-0.7/3)
 *   errp^(0.4/3) within [0.2, 5] h ([0.2, 1] h after a rejection, errp the last
 *   accepted err, at least 1e-4), rejected steps retried with
 *   h max(0.2, 0.9 err^(-1/3)); the last step ends exactly at t_end.
 * Advances q (device state, context dtype) in place from t0 to t_end with a
 * first attempted step dt0.  adaptive = 0: fixed steps dt0, all accepted (the
 * estimate is still formed and recorded).  At most max_attempts attempts (then
 * out->reached_end = 0).  record (device, may be NULL when record_cap = 0):
 * (h, err, accepted) of attempt n at record[3n .. 3n+2] for n < record_cap.
 * Error norms and the controller run on the device (FP64 whatever the dtype);
 * attempts are replayed from a captured graph and the host looks at the run
 * state once every 32 attempts.  SGN_OPT_STEP_PATH picks the kernels of an
 * attempt: on SGN_PATH_FUSED (default) the four evaluations after k_1 run in
 * one launch of the step kernel's tile (the stages stay in LDS), on the other
 * paths as four stage kernels; the same bits either way.  Uses three more
 * state-sized buffers (two k_1 and the error estimate), allocated on first use
 * and kept by the context.  Synchronizes.  Errors: SGN_E_ARG
 * (t_end < t0, dt0 <= 0, negative or zero tolerances, max_attempts < 1),
 * SGN_E_UNSUPPORTED with a source term, SGN_E_NONFINITE when an error norm is
 * not finite, SGN_E_NONPOS_DEPTH when an accepted step leaves h <= 0 (q then
 * holds the last accepted state; out is filled in every case after the
 * arguments are checked). */
sgn_status sgn_step_adaptive(sgn_ctx* ctx, void* q, double t0, double t_end, double dt0, double rtol, double atol,
                             int32_t adaptive, int64_t max_attempts, double* record, int64_t record_cap,
                             sgn_adaptive_result* out);

/* Total mass 1^T M h (FP64 result, compensated deterministic summation). */
sgn_status sgn_mass(sgn_ctx* ctx, const void* q, double* out);

/* Total energy 1^T M E with E = h((u^2+v^2)/2 + w^2/6 + g/2 (h+2b)
 * + lambda/6 (eta/h - 1)^2) (FP64 result). */
sgn_status sgn_energy(sgn_ctx* ctx, const void* q, double* out);

/* Both totals in one pass. */
sgn_status sgn_mass_energy(sgn_ctx* ctx, const void* q, double* mass, double* energy);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the totals of
 * sgn_mass_energy without a context.  Same kernels, so the same bits as
 * sgn_mass_energy on a context with these params and bathymetry.
 *   params: validated like sgn_create (source ignored); q: device state
 *   (5 planes, params->dtype); b: device bathymetry plane (params->dtype);
 *   stream: hipStream_t (NULL for the null stream); out: device memory of two
 *   doubles, receives mass and energy (FP64 whatever the dtype).
 * Asynchronous on stream; allocates nothing: the partial sums go to a static
 * device array of 32 KiB that each GPU holds until the process ends (every grid
 * size fits), looked up once per device on the first call there.  Calls that
 * overlap on one GPU (different streams or threads) share that array and race:
 * order them.  Errors: SGN_E_ARG / SGN_E_SHAPE as sgn_create or for NULL
 * pointers, SGN_E_HIP for launch failures; the message is left for
 * sgn_last_error(NULL). */
sgn_status sgn_mass_energy_noalloc(const sgn_params* params, const void* q, const void* b, void* stream,
                                   double* out);

/* Semi-discrete rates 1^T M h_t and <d_q E, q_t>_M (Theorem 1 proof); both
 * vanish up to rounding for any state with h > 0.  Uses the context's scratch. */
sgn_status sgn_rates(sgn_ctx* ctx, const void* q, double* mass_rate, double* energy_rate);

/* dt = cfl / max_ij [(|u|+c)/dx + (|v|+c)/dy] with c^2 = g h + lambda eta^2/(3 h^2). */
sgn_status sgn_cfl_dt(sgn_ctx* ctx, const void* q, double cfl, double* dt);

/* Measurement: advance q by nsteps RK4 steps like sgn_step but with direct
 * launches, recording HIP events on the context's stream (all enqueued before
 * the first wait, so the kernels run back to back).  Four-stage path: an event
 * between consecutive kernels, ms[s] = mean duration of stage kernel s (0 =
 * first, 1 and 2 = middle, 3 = last).  Pair path: likewise, ms[0] = pair 1,
 * ms[1] = pair 2, ms[2] = ms[3] = 0.  Fused path (one kernel per step): a start
 * and a stop event bound to each step kernel's own execution, nothing enqueued
 * between the launches; ms[0] = the step kernel, ms[1..3] = 0.  On
 * the pair and fused paths an odd nsteps is rounded up; the means leave out
 * the first step (two on those paths) when there are more.  nsteps <= 1024
 * (SGN_E_ARG otherwise).  Milliseconds; synchronizes. */
sgn_status sgn_profile_stages(sgn_ctx* ctx, void* q, double dt, int64_t nsteps, double* ms);

/* Synchronize and report (then clear) the device health flag. */
sgn_status sgn_check(sgn_ctx* ctx);

/* Grid spacing used by the context (host doubles). */
sgn_status sgn_spacing(const sgn_ctx* ctx, double* dx, double* dy);

/* ------------------------------------------------------------------------
 * Discrete adjoint (vector-Jacobian products of the semi-discretization and
 * of the RK4 step, differentiated after discretization).  Defined without
 * source terms (SGN_E_UNSUPPORTED otherwise).  Work buffers are allocated on
 * first use and owned by the context until sgn_destroy.
 * ------------------------------------------------------------------------ */

/* (qbar, bbar) = J^T a, J the Jacobian of sgn_rhs at q with respect to (q, b).
 * a, qbar: states; bbar: one plane.  Overwrites qbar and bbar. */
sgn_status sgn_rhs_vjp(sgn_ctx* ctx, const void* q, const void* a, void* qbar, void* bbar);

/* Reverse of one RK4 step of size dt from q_n.  On entry qbar holds the
 * cotangent of q_{n+1}; on exit the cotangent of q_n.  bbar accumulates (+=)
 * the bathymetry cotangent.  The stage states are recomputed (by the pair
 * kernels on SGN_PATH_PAIRS, by the step kernel otherwise; the same values
 * either way) and reversed in the order k4, k3, k2, k1: on SGN_PATH_FUSED
 * (default) two stages per launch (k4 with k3, k2 with k1), on the other
 * paths one stage per launch; the two forms agree to rounding. */
sgn_status sgn_step_vjp(sgn_ctx* ctx, const void* q_n, double dt, void* qbar, void* bbar);

/* Gauge series of a rollout: from the initial surface zeta0 (device plane),
 * h0 = zeta0 - b, u0 = v0 = 0, eta0 = h0 and w0 by eq. (initialization),
 * advance nsteps RK4 steps of size dt and record zeta = h + b at the gauge
 * nodes gauge_idx[g] (device int64 row-major node indices, 1..4096 gauges)
 * after every step into series[n * ngauges + g] (device doubles, n = 0 is the
 * state after the first step).  Synchronizes. */
sgn_status sgn_gauge_series(sgn_ctx* ctx, const void* zeta0, int64_t nsteps, double dt, const int64_t* gauge_idx,
                            int32_t ngauges, double* series);

/* Loss L = 1/2 sum_n sum_g (zeta_g^n - target[n * ngauges + g])^2 over the
 * rollout of sgn_gauge_series (target: device doubles) and its gradient with
 * respect to the initial surface (grad_zeta0) and the bathymetry (grad_b),
 * both device planes.  The forward rollout stores a checkpoint every
 * checkpoint_every steps (0: ceil(sqrt(nsteps))); the reverse sweep
 * recomputes one segment at a time, keeping its states and stage states, and
 * runs the step VJPs backwards.  The forward steps follow the context's step
 * path (pair kernels on SGN_PATH_PAIRS, the step kernel otherwise), and so do
 * the step VJPs (as in sgn_step_vjp).  Memory: checkpoints plus 4*K+1 states
 * for a segment of K steps, plus five states of cotangent work buffers.  With
 * SGN_OPT_ADJOINT_STORE = B bytes the forward rollout itself keeps the states
 * and stage states of its last F = min(nsteps, (B / S - 1) / 4) steps (S the
 * bytes of one state; 4*F+1 states, the same storage the segments reuse
 * afterwards), the reverse sweep reverses those without recomputing them, and
 * the checkpoints and segments cover the first nsteps - F steps only
 * (checkpoint_every 0: ceil(sqrt(nsteps - F))).  Loss and gradients are the
 * same bit for bit whatever B.  *loss is a host double.  Synchronizes.
 * Errors: SGN_E_ALLOC when the storage cannot be allocated. */
sgn_status sgn_gauge_loss_grad(sgn_ctx* ctx, const void* zeta0, int64_t nsteps, double dt, const int64_t* gauge_idx,
                               int32_t ngauges, const double* target, int64_t checkpoint_every, double* loss,
                               void* grad_zeta0, void* grad_b);

/* ------------------------------------------------------------------------
 * Ensembles: many independent problems advanced together.
 *
 * Every instance has its own sgn_params (grid size, domain, boundary types, g,
 * lambda; all instances share one dtype; no source terms) and its own time
 * step.  The tiles of all instances form one work list; each RK4 step is one
 * launch running the step tile of SGN_PATH_FUSED over the whole list
 * (default), or two launches running the stage-pair tiles of SGN_PATH_PAIRS;
 * the boundary variant is chosen per instance.  A launch has one workgroup
 * per tile (default) or a persistent grid (sgn_batch_set_tiling).  Steps are
 * replayed from a captured HIP graph.  Results are identical, bit for bit, to
 * advancing each instance alone with sgn_step (every step path forms the same
 * values).
 *
 * The caller owns the states (n device pointers, each 5 planes of that
 * instance's ny*nx values in the batch dtype) and passes them with
 * sgn_batch_set_states; the batch owns packed copies of the bathymetries, the
 * scratch states and per-instance health flags.  Synchronization, errors and
 * threading follow the single-problem rules above.
 * ------------------------------------------------------------------------ */
typedef struct sgn_batch sgn_batch;

sgn_status sgn_batch_create(int32_t n, const sgn_params* params, void* stream, sgn_batch** out);
sgn_status sgn_batch_destroy(sgn_batch* batch);
/* Copy instance i's bathymetry (device plane of its ny*nx values). */
sgn_status sgn_batch_set_bathymetry(sgn_batch* batch, int32_t i, const void* b);
/* Register the n state pointers (q[i] device, caller-owned, not copied). */
sgn_status sgn_batch_set_states(sgn_batch* batch, void* const* q);
/* eq. (initialization) on every state in place. */
sgn_status sgn_batch_init_aux(sgn_batch* batch);
/* Advance every instance by nsteps RK4 steps; dt is a host array of n steps. */
sgn_status sgn_batch_step(sgn_batch* batch, const double* dt, int64_t nsteps);
/* Per-instance totals into host arrays of n doubles (either may be NULL).  Synchronizes. */
sgn_status sgn_batch_mass_energy(sgn_batch* batch, double* mass, double* energy);
/* Per-instance CFL steps (rule of sgn_cfl_dt) into a host array of n doubles.  Synchronizes. */
sgn_status sgn_batch_cfl_dt(sgn_batch* batch, double cfl, double* dt);
/* SGN_PATH_FUSED (default) or SGN_PATH_PAIRS (SGN_E_UNSUPPORTED otherwise).
 * Resets the tile height to the path's default (fused: 24; pairs: 8 in SGN_F64,
 * 16 in SGN_F32). */
sgn_status sgn_batch_set_step_path(sgn_batch* batch, int32_t path);
/* Tile height (8 or 16, and 24 on the fused path; there 8 selects 64 x 8
 * tiles, 16 selects 32 x 16 and 24 selects 32 x 24) and persistent
 * workgroups per compute unit (1..16), or 0 for one workgroup per tile (the
 * default: no persistent loop, fewer registers; the only choice for 32 x 24,
 * SGN_E_UNSUPPORTED otherwise). */
sgn_status sgn_batch_set_tiling(sgn_batch* batch, int32_t tile_y, int32_t blocks_per_cu);
/* Time every (tile height 8, 16 or 24 (fused path, one workgroup per tile),
 * 0..6 workgroups per CU) candidate of the
 * current step path on one step from the
 * registered states into scratch (the states are read, never written), keep
 * the fastest and report it (any output may be NULL; ms = time of one step).
 * Synchronizes. */
sgn_status sgn_batch_autotune(sgn_batch* batch, const double* dt, int32_t* tile_y, int32_t* blocks_per_cu,
                              double* ms);
/* Synchronize; report (and clear) health flags; *first_bad = first failing instance or -1. */
sgn_status sgn_batch_check(sgn_batch* batch, int32_t* first_bad);
/* Sum of nx*ny over the instances. */
sgn_status sgn_batch_total_nodes(const sgn_batch* batch, int64_t* nodes);
const char* sgn_batch_last_error(const sgn_batch* batch);

/* Message of the last failed call on ctx (or of the last failed sgn_create when ctx is NULL). */
const char* sgn_last_error(const sgn_ctx* ctx);

/* Static name of a status code. */
const char* sgn_status_string(int32_t status);

#ifdef __cplusplus
}
#endif

#endif /* SGN_H */
