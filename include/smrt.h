/*
 * smrt.h -- C ABI of the MI355X (gfx950) Second Moment thermal radiative
 * transfer library: the lumped DG S_N transport sweep with fused angular
 * moments, the SM closures, the FP64 low-order solve and one backward-Euler
 * step, following Olivier, Warsa & Park, "Efficient, Nonlinear Second
 * Moment Methods for Multigroup Thermal Radiative Transfer".
 *
 * General rules
 *  - Every call returns an smrt_status and never throws.  On failure the
 *    message is available from smrt_last_error(ctx) (a thread-local copy
 *    for calls that fail before a context exists: smrt_last_error(NULL)).
 *  - Host arrays passed in are copied; the caller may free them after the
 *    call returns.  Arrays written by the library are caller-owned buffers
 *    of the documented size.
 *  - "_dev" entry points take device pointers (e.g. from torch) that the
 *    library borrows for the duration of the call only; work is ordered on
 *    the context's HIP stream and the call returns after the stream is
 *    synchronised unless stated otherwise.
 *  - The context owns every device buffer it allocates (angular flux ping-
 *    pong, moments, low-order operators, traces, scratch) and frees them in
 *    smrt_destroy.
 *
 * Discretisation and numbering (Sec. 3 of the paper; all forms lumped with
 * the trapezoid rule, Sec. 6):
 *  - rectilinear mesh, nx (x ny) cells; cell c = i + nx*j;
 *  - bilinear (2D) / linear (1D) DG nodes at the cell vertices; local node
 *    l = lx + 2*ly; node n = 2^dim * c + l; every nodal array uses n;
 *  - angular arrays in the ABI ("psi") are laid out [d][g][node];
 *  - boundary face nodes (general inflow arrays): 1D x-=0, x+=1; 2D: x- side
 *    2j+ly, x+ side 2ny+2j+ly, y- side 4ny+2i+lx, y+ side 4ny+2nx+2i+lx.
 *  - moment arrays ([27][node] in 2D, [8][node] in 1D), FP64: 2D quadrant
 *    q (0:(mu>0,eta>0) 1:(mu<0,eta>0) 2:(mu<0,eta<0) 3:(mu>0,eta<0)) at rows
 *    6q+k, k = sums over d in q and all g of w*{1,mu,eta,mu^2,mu*eta,eta^2}*I;
 *    rows 24..26 = sum_g sigma_g sum_d w*{1,mu,eta}*I.  1D: half h (0:mu>0,
 *    1:mu<0) at rows 3h+k for w*{1,mu,mu^2}*I; rows 6,7 = sigma-weighted
 *    {1, mu}.
 */
#ifndef SMRT_H
#define SMRT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct smrt_ctx smrt_ctx;
typedef struct smrt_batch smrt_batch;

typedef enum {
    SMRT_OK = 0,
    SMRT_E_INVALID_ARG = 1,
    SMRT_E_OUT_OF_MEMORY = 2,
    SMRT_E_DEVICE = 3,
    SMRT_E_NOT_CONVERGED = 4,
    SMRT_E_NONPHYSICAL = 5,
    SMRT_E_STATE = 6
} smrt_status;

/* Precision of the sweep and of the stored angular flux.  The low-order
 * solve, closures and energy balance always run in FP64. */
typedef enum { SMRT_FP64 = 0, SMRT_FP32 = 1 } smrt_precision;

/* Low-order scheme: consistent LDG SM (Sec. 4), independent LDG SM (Sec. 4),
 * or the unaccelerated sweep + pointwise elimination iteration (Sec. 6). */
typedef enum { SMRT_SM_CONSISTENT = 0, SMRT_SM_INDEPENDENT = 1, SMRT_UNACCELERATED = 2 } smrt_scheme;

/* Rectilinear mesh.  dim = 1 or 2; x_edges[nx+1] strictly increasing;
 * y_edges[ny+1] in 2D (ny = 1 and y_edges = NULL in 1D). */
typedef struct {
    int dim, nx, ny;
    const double *x_edges, *y_edges;
} smrt_mesh_desc;

/* Discrete ordinates {Omega_d, w_d} (Sec. 2): omega[n][3] unit vectors,
 * w[n] with sum w = 4*pi (|sum - 4pi| <= 1e-12*4pi); no direction may have
 * mu = 0, nor eta = 0 in 2D.  1D uses omega[d][0] = mu only. */
typedef struct {
    int n_angles;
    const double *omega;
    const double *w;
} smrt_quad_desc;

/* Groups (Sec. 2): nu_edges[G+1] strictly increasing stated group bounds.
 * The Planck/Rosseland fractions integrate the first group from 0 and the
 * last group to infinity, so that sum_g b_g = 1.  a = radiation constant,
 * c = speed of light. */
typedef struct {
    int G;
    const double *nu_edges;
    double a, c;
} smrt_groups_desc;

/* Materials.  model 0: sigma_g = sigma0[r*G+g] (constant); model 1:
 * sigma_g = sigma0[r] / (nubar_g^3 T_cell^3) clipped to [clip_lo, clip_hi],
 * nubar_g = sqrt(nu_g nu_{g+1}) and T_cell the mean of the cell's nodal
 * temperatures (Sec. 3: piecewise-constant opacity from the element-average
 * temperature).  cv[r] = heat capacity of region r. */
typedef struct {
    int n_regions;
    const int32_t *region_of_cell;
    int model;
    const double *sigma0;
    double clip_lo, clip_hi;
    const double *cv;
} smrt_material_desc;

/* Boundary, per side (1D: x-, x+; 2D: x-, x+, y-, y+): kind 0 vacuum,
 * 1 isotropic Planck inflow B_g(T_bdr)/(4 pi), 2 explicit isotropic inflow
 * inflow_g[side][g] (intensity per group), 3 reflective (specular: the
 * symmetry planes of Sec. 6).  On a reflective side a direction entering
 * the domain takes, at each boundary node, the intensity of its mirror
 * image (mu -> -mu on x sides, eta -> -eta on y sides) at that node: the
 * context refreshes it from the newest intensity (smrt_set_state, after
 * every sweep of a step or resident pass), and the closures take that
 * inflow's incoming moments node by node.  Kind 3 needs the mirror image of
 * every direction, with the same weight, in the quadrature
 * (SMRT_E_INVALID_ARG otherwise). */
typedef struct {
    int kind[4];
    double T_bdr[4];
    const double *inflow_g[4];
} smrt_boundary_desc;

/* Iteration control (Sec. 6 defaults: eps 1e-3, CG and elimination rtol
 * 1e-10, caps 100/30/50/40).  strict = 1 turns a capped iteration into
 * SMRT_E_NOT_CONVERGED.  fixed_outer > 0 runs exactly that many outer
 * iterations (used to replay a reference iteration count). */
typedef struct {
    double eps_outer, eps_inner, cg_rtol, elim_rtol;
    int max_outer, max_inner, max_cg, max_elim;
    smrt_precision precision;
    smrt_scheme scheme;
    int strict;
    int fixed_outer;
    int lo_time_edge;   /* 0: E*, F* = HO sums of I^k (default); 1: LO solution */
    int lo_graphs;      /* 1 (default): the LO conjugate-gradient iterations replay a captured HIP
                           graph of 4 iterations; 0: launched one kernel at a time */
    int fixup;          /* 1: zero-and-scale negative-flux fixup inside every sweep (Sec. 6, after
                           Hamilton et al.): a cell whose solution has a negative entry gets those
                           entries set to 0 and the others scaled by one factor that keeps the
                           cell's particle balance (the sum of the rows of its local system); a
                           cell whose balance has a non-positive right side is set to 0.
                           0 (default): the plain linear sweep */
    double T_floor;     /* > 0: temperature floor (Sec. 6): the pointwise energy balance returns
                           max(root, T_floor), and T_floor where it has no positive root, instead
                           of failing with SMRT_E_NONPHYSICAL.  0 (default): no floor.  In the
                           problem's temperature units. */
    int lo_precond;     /* preconditioner of the LO conjugate gradients (Sec. 5 solves them with an
                           algebraic-multigrid preconditioner): 0 (default) Jacobi; 1 aggregation
                           multigrid (cells, then 2x2 blocks of cells, Galerkin coarse operators,
                           damped-Jacobi smoothing, one V-cycle per iteration), rebuilt for every
                           Newton linearisation.  Changes the iteration count, not the solution. */
} smrt_options;

/* Per-step statistics (the columns of the paper's summary tables). */
typedef struct {
    int outer, inner_total, cg_total, elim_max, hit_max;
    double t_sweep_ms, t_lo_ms, t_total_ms;
} smrt_step_stats;

/* Fills *o with the paper's defaults (FP64, consistent SM). */
void smrt_default_options(smrt_options *o);

/* Creates a problem context.  Validates every descriptor (see the struct
 * comments; SMRT_E_INVALID_ARG on violation), copies them, allocates all
 * device memory (SMRT_E_OUT_OF_MEMORY), builds the low-order operators, and
 * sets the state to the isotropic equilibrium of T = 0 (call
 * smrt_set_state next).  hip_stream: a hipStream_t to order all work on, or
 * NULL for a stream owned by the context.  Requires a gfx950 device. */
smrt_status smrt_create(const smrt_mesh_desc *mesh, const smrt_quad_desc *quad, const smrt_groups_desc *groups,
                        const smrt_material_desc *mat, const smrt_boundary_desc *bc, const smrt_options *opt,
                        void *hip_stream, smrt_ctx **out);

void smrt_destroy(smrt_ctx *ctx);

/* Last error message of ctx (or of the calling thread when ctx is NULL). */
const char *smrt_last_error(const smrt_ctx *ctx);

/* Replaces iteration options (precision cannot change after create). */
smrt_status smrt_set_options(smrt_ctx *ctx, const smrt_options *opt);

/* Replaces the boundary description (e.g. per-step T_bdr). */
smrt_status smrt_set_boundary(smrt_ctx *ctx, const smrt_boundary_desc *bc);

/* Sets the state: T_nodes[n_nodes] (finite, > 0) and psi[d][g][node] (FP64;
 * rounded to the context precision) or NULL for the isotropic equilibrium
 * B_g(T)/(4 pi) (problems start in equilibrium).  The low-order E is set to
 * the HO energy density of psi and F to its flux. */
smrt_status smrt_set_state(smrt_ctx *ctx, const double *T_nodes, const double *psi);

/* Copies out T[n_nodes], E[n_nodes] (low-order energy density), F[dim*n]
 * (low-order flux, node-major) and, if psi != NULL, the angular flux
 * [d][g][node] (FP64).  Any pointer may be NULL. */
smrt_status smrt_get_state(smrt_ctx *ctx, double *T, double *E, double *F, double *psi);

/* Raw sweep (Eq. dgsn_transport, lumped): for every (d, g) solves
 *   Omega.grad I + sigt I = q_iso + inv_c_dt * psi_prev
 * with upwind traces, in downstream order, and accumulates the moments.
 * sig_t[cell][G] total (incl. time absorption) and sig[cell][G] absorption
 * opacities (the latter weights rows 24..26 / 6..7 of the moments);
 * q_iso[node][G]; psi_prev [d][g][node] or NULL (zero); psi_inflow general
 * inflow [d][g][boundary node] or NULL (use the boundary description; a
 * reflective side then carries the mirror of the context's last intensity:
 * this call sweeps once and does not iterate the reflection).
 * Host arrays are in FP64; psi_out ([d][g][node], FP64, may be NULL) and
 * moments_out ([27 or 8][node], FP64, may be NULL) are written.  The sweep
 * itself runs at the context precision. */
smrt_status smrt_sweep(smrt_ctx *ctx, const double *sig_t, const double *sig, const double *q_iso,
                       const double *psi_prev, double inv_c_dt, const double *psi_inflow, double *psi_out,
                       double *moments_out);

/* smrt_sweep on device arrays (e.g. torch tensors): the same operation
 * (Sec. 3, eq. dgsn_transport, lumped) and the same layouts, all FP64 and
 * contiguous, but every pointer is a device address on the context's GPU.
 * The arrays are borrowed for the duration of the call and never freed;
 * the work is ordered on the context stream (the caller makes the inputs
 * ready on it, e.g. by creating the context on its own stream or
 * synchronizing first) and the call returns once the outputs are written.
 * psi_out ([d][g][node]) is required; psi_prev, psi_inflow and moments_out
 * may be NULL as in smrt_sweep.  Errors: SMRT_E_INVALID_ARG for a NULL
 * required array, inv_c_dt < 0 or not finite, or (checked on the device)
 * sig_t <= 0 or sig < 0 anywhere. */
smrt_status smrt_sweep_dev(smrt_ctx *ctx, const double *sig_t, const double *sig, const double *q_iso,
                           const double *psi_prev, double inv_c_dt, const double *psi_inflow, double *psi_out,
                           double *moments_out);

/* smrt_sweep_dev for callers that cannot allocate device memory (serving
 * loops, harnesses that forbid hipMalloc): the same operation, arguments,
 * layouts and errors, but every per-call work array (inputs in the sweep's
 * internal layouts, the internal output, moment partials, band trace words,
 * counters) lives in one static device array of 64 MiB that each GPU the
 * library runs on holds until the process ends; the call makes no
 * allocation.  Problems whose work arrays exceed 64 MiB are rejected with
 * SMRT_E_INVALID_ARG (the message gives the bytes needed): use
 * smrt_sweep_dev for them.  The call waits for the context stream before it
 * returns.  All calls on one GPU share its array, which keeps the last
 * call's contents: calls that overlap on one GPU (from several threads or
 * streams) race and must be serialised by the caller. */
smrt_status smrt_sweep_dev_static(smrt_ctx *ctx, const double *sig_t, const double *sig, const double *q_iso,
                                  const double *psi_prev, double inv_c_dt, const double *psi_inflow, double *psi_out,
                                  double *moments_out);

/* Adjoint sweep: the transpose of the lumped upwind DG transport operator
 * of smrt_sweep (Sec. 3, eq. dgsn_transport), the building block of the
 * adjoint of a time step.  For every (d, g):
 *   lambda_d = L_d^{-T} (w . src_d),
 * L_d the sweep operator of direction d for total cross section
 * sig_t[cell][G] (> 0) with zero inflow (the adjoint boundary condition is
 * homogeneous), w the lumped nodal weights |cell| / 2^dim.  src and
 * lambda_out are [d][g][node] FP64.  If dsig_out ([cell][G], may be NULL)
 * is given, emis ([node][G], emission per unit opacity B_g/4pi) and psi_fwd
 * ([d][g][node], the forward intensity) are required and
 *   dsig_out[c][g] = sum_d sum_{l in c} w_l lambda_{d,g,l} (emis_{l,g} - psi_fwd_{d,g,l}),
 * the derivative of <lambda, transport residual> with respect to sigma_g of
 * the cell through the emission and removal terms (with the sign of a
 * gradient of J when lambda solves the adjoint of dJ/dI).  Needs a quadrature
 * closed under Omega -> -Omega (level-symmetric, Gauss-Legendre); runs at
 * the context precision.  Errors: SMRT_E_INVALID_ARG for NULL inputs,
 * sig_t <= 0 or a quadrature without opposite directions. */
smrt_status smrt_adjoint_sweep(smrt_ctx *ctx, const double *sig_t, const double *src, const double *emis,
                               const double *psi_fwd, double *lambda_out, double *dsig_out);

/* Replace the per-region material parameters (Sec. 2 opacity and heat
 * capacity): sigma0 as given to smrt_create ([n_regions] for the power-law
 * model, [n_regions][G] for constant opacities) and cv[n_regions]; either
 * may be NULL to keep it.  Copied.  Errors: SMRT_E_INVALID_ARG for negative
 * sigma0, non-positive cv or both NULL. */
smrt_status smrt_set_materials(smrt_ctx *ctx, const double *sigma0, const double *cv);

/* Adjoint gradient (the differentiable form of the time step).  From the
 * context's current state, runs n_steps backward-Euler steps of length dt
 * (smrt_step with the context options; use tight tolerances so each step is
 * at its fixed point), keeping per-step checkpoints of I, T and sigma, and
 * returns the objective
 *   0: the time-integrated outflow through the x+ boundary,
 *      J = sum_k dt sum_g sum_{mu_d > 0} w_d mu_d sum_{n on x+} fw_n I^k_{d,g,n};
 *   1: the material energy at the last step, J = sum_n w_n c_v,n T^N_n
 *      (w_n the lumped nodal weight),
 * with its gradient with respect to log sigma0_r and log c_v,r (grad arrays
 * [n_regions]; for objective 1 the c_v gradient includes J's direct
 * dependence on c_v).  The gradient is
 * that of the converged discrete solution of every step (transport with
 * emission, Sec. 3, plus the lumped energy balance, Sec. 2), obtained
 * backwards by adjoint source iteration: adjoint sweeps (smrt_adjoint_sweep)
 * alternating with the pointwise temperature adjoint.  Clipped opacities
 * contribute no sigma0 sensitivity.  adjoint_iterations (may be NULL)
 * receives the total number of adjoint source iterations.  The context
 * state is advanced by n_steps.  Errors: SMRT_E_INVALID_ARG (objective not
 * 0 or 1, n_steps < 1, dt <= 0, constant-opacity model, quadrature without
 * opposite directions, no state, fixup or T_floor switched on: the adjoint is
 * that of the linear sweep and the unfloored balance, a reflective side), or
 * the failure of a forward step. */
smrt_status smrt_adjoint(smrt_ctx *ctx, int objective, int n_steps, double dt, double *J, double *grad_log_sigma0,
                         double *grad_log_cv, int *adjoint_iterations);

/* Closures and low-order sources (Sec. 2 gray collapse, Sec. 4 consistent /
 * independent LDG sources) from HO moments (FP64 [27|8][node], as produced by
 * smrt_sweep), the outer-iterate temperature T_l[n], the time-edge sources
 * Estar[n], Fstar[dim*n], the absorption opacity sig[cell][G], and dt.
 * Output closures_out [5+dim... ] laid out as rows [sigE, sigF, sigP, qE,
 * qF_x(, qF_y)] x n_nodes.  Uses the context's boundary description and
 * scheme; a reflective side takes the context's current reflected inflow
 * (the mirror of the last intensity the context swept or was given). */
smrt_status smrt_compute_closures(smrt_ctx *ctx, const double *moments, const double *T_l, const double *Estar,
                                  const double *Fstar, const double *sig, double dt, double *closures_out);

/* Low-order Newton solve with nonlinear elimination (Sec. 5) for fixed
 * closures (rows as produced by smrt_compute_closures), time-edge
 * temperature Tstar[n] and dt: E[n], T[n] in (initial guess) / out, F[dim*n]
 * out.  Stats: inner_total, cg_total, elim_max, hit_max. */
smrt_status smrt_lo_solve(smrt_ctx *ctx, const double *closures, const double *Tstar, double dt, double *E,
                          double *F, double *T, smrt_step_stats *stats);

/* One backward-Euler step of length dt (Algorithm 1) from the context's
 * current state; all data stays on the device. */
smrt_status smrt_step(smrt_ctx *ctx, double dt, smrt_step_stats *stats);

/* Resident high-order pass, for throughput measurement: n_times times, on
 * the context's current state (T, psi as psi_prev) with time step dt, runs
 * the opacity table, the emission source and gray-collapse tables, the
 * sweep with fused moments, the moment finalisation and the closure
 * post-pass, all on the context stream with no host transfer.  Writes the
 * mean wall time per pass (ms) and the mean duration of the sweep kernel
 * alone (ms), both measured with HIP events on the context stream.  The
 * state (T, psi) is not advanced. */
smrt_status smrt_sweep_resident(smrt_ctx *ctx, double dt, int n_times, double *ms_per_pass, double *ms_sweep_kernel);

/* Copies the HO moments of the most recent sweep of the context (the last
 * outer iteration of smrt_step, or smrt_sweep_resident) into moments
 * ([27|8][n_nodes], FP64, layout as in the header comment). */
smrt_status smrt_get_moments(smrt_ctx *ctx, double *moments);

/* Information about the problem and the chosen launch configuration. */
typedef struct {
    int dim, nx, ny, n_angles, G, n_nodes, n_cells;
    int64_t units_per_sweep;
    int64_t algorithmic_bytes_per_sweep;   /* read I* + write I, at the sweep precision */
    int band_rows, waves_per_band, pairs_per_lane, pairs_per_chunk, n_chunks, n_workgroups;
    int bands_per_group;
} smrt_info;
smrt_status smrt_get_info(const smrt_ctx *ctx, smrt_info *info);

/* Sweep launch configuration override (2D; 0 = automatic per field).  A
 * sweep workgroup sweeps one direction and a block of groups on a group of
 * consecutive bands of 16 rows: waves_per_band in {0, 1, 2, 4} waves share
 * a band (4 pairs_per_lane groups each), bands_per_group in {0, 1, 2, 4,
 * 8, 16} bands run in lockstep in one workgroup (the band hand-off goes
 * through LDS), at most 16 waves in all; pairs_per_lane in {0, 1, 2, 4}
 * (4: FP32 only).  Automatic: one wave per band, one group per lane, and
 * the fewest bands (a power of two) that cover the mesh within 16 waves.
 * Returns SMRT_E_INVALID_ARG outside these ranges. */
smrt_status smrt_set_launch(smrt_ctx *ctx, int waves_per_band, int bands_per_group, int pairs_per_lane);

/* Name of the current HIP device and its architecture ("<name> <gcnArch>",
 * truncated to len - 1 characters and NUL-terminated) and its compute-unit
 * count: the key under which tuned launch shapes are cached.  Errors:
 * SMRT_E_INVALID_ARG for a NULL buffer or len < 1, SMRT_E_DEVICE. */
smrt_status smrt_device_name(char *buf, int len, int *n_compute_units);

/* Sweep occupancy (2D): at most workgroups_per_cu sweep workgroups share a
 * compute unit (the launch pads its LDS request accordingly); 0 = as many as
 * the registers allow (default).  Errors: SMRT_E_INVALID_ARG outside [0, 8]. */
smrt_status smrt_set_occupancy(smrt_ctx *ctx, int workgroups_per_cu);

/* Launch-shape autotuner (2D): on the context's current state with time step
 * dt, times one sweep for every candidate (waves per band, bands per
 * workgroup, groups per lane) whose chunk covers less than twice the groups
 * and whose workgroup less than twice the bands of the problem, each at
 * occupancy 0, 1 and 2 workgroups per CU, applies the fastest and returns its
 * shape, its occupancy (as smrt_set_occupancy takes it) and its sweep time in
 * ms (any output pointer may be NULL).  The state is not advanced.  Errors:
 * SMRT_E_INVALID_ARG before smrt_set_state, for 1D, or for dt <= 0. */
smrt_status smrt_autotune(smrt_ctx *ctx, double dt, int *waves_per_band, int *bands_per_group, int *pairs_per_lane,
                          int *workgroups_per_cu, double *ms_best);

/* ---- Batches: many independent 2D problems swept in one launch ---------
 * A batch borrows n contexts (all 2D, one precision, each with a state) and
 * sweeps every (problem, chunk, band group) task of all of them in one
 * launch, in an order where every band group follows the group below it of
 * the same problem (no deadlock at any residency) and the longest bands
 * start first.  The contexts stay
 * owned by the caller and must outlive the batch; the batch re-plans their
 * sweep launch shape (one shape for the whole batch).  A batch call drains
 * every problem's stream, works on the batch's own stream and drains it
 * before returning.  The LO of each
 * problem stays per problem, in FP64 (Sec. 5). */
typedef struct smrt_batch smrt_batch;
smrt_status smrt_batch_create(int n, smrt_ctx *const *problems, smrt_batch **out);
void smrt_batch_destroy(smrt_batch *batch);
const char *smrt_batch_last_error(const smrt_batch *batch);
/* Launch shape shared by the batch (as smrt_set_launch, every field given:
 * no automatic value). */
smrt_status smrt_batch_set_launch(smrt_batch *batch, int waves_per_band, int bands_per_group, int pairs_per_lane);
/* Occupancy of the batched sweep (as smrt_set_occupancy). */
smrt_status smrt_batch_set_occupancy(smrt_batch *batch, int workgroups_per_cu);
/* Total units per batched sweep, workgroup tasks, and the launch shape. */
smrt_status smrt_batch_info(const smrt_batch *batch, int64_t *units_per_sweep, int *n_tasks, int *waves_per_band,
                            int *bands_per_group, int *pairs_per_lane);
/* Batch autotuner: times the batched sweep for every candidate launch shape
 * and occupancy on the problems' current states with time step dt, applies
 * and returns the fastest (shape, occupancy, ms of one batched sweep). */
smrt_status smrt_batch_autotune(smrt_batch *batch, double dt, int *waves_per_band, int *bands_per_group,
                                int *pairs_per_lane, int *workgroups_per_cu, double *ms_best);
/* Resident high-order pass of every problem (as smrt_sweep_resident, with
 * all sweeps in one batched launch), n_times.  capture_graph != 0 records
 * the pass once as a HIP graph (kernels only) and replays it n_times.
 * Writes the mean time per pass and the time of one batched sweep launch
 * (ms).  States are not advanced. */
smrt_status smrt_batch_sweep_resident(smrt_batch *batch, double dt, int n_times, int capture_graph,
                                      double *ms_per_pass, double *ms_sweep_kernel);
/* One backward-Euler step (Algorithm 1) of every problem, dt[n] per problem:
 * the outer iterations run in lock-step, each with one batched sweep over
 * the problems still iterating; stats[n] (may be NULL) per problem.  Returns
 * the first problem's failure status (message in smrt_batch_last_error). */
smrt_status smrt_batch_step(smrt_batch *batch, const double *dt, smrt_step_stats *stats);
/* n_steps backward-Euler steps (Algorithm 1) of every problem with the
 * convergence decisions on the device: each problem's outer iteration is
 * stopped by its own test (Algorithm 1: eps_outer, fixed_outer, max_outer)
 * in a control block in device memory, and its LO solve (Sec. 5: Newton
 * with nonlinear elimination, Jacobi-preconditioned CG, their tests and
 * caps) runs for all problems in one persistent launch whose workgroups
 * meet at grid barriers.  The host queues blocks of 4 outer iterations of
 * the whole batch (one batched sweep each; a converged problem skips the
 * rest of them) and waits once per block, and once per step;
 * capture_graph != 0 records the block once as a HIP graph and replays it.
 * dt[n_steps * n]: step s of problem p at dt[s * n + p]; stats (may be NULL)
 * [n_steps * n] likewise (t_total_ms: the whole batch's step; t_sweep_ms and
 * t_lo_ms are not separated: 0).  Each problem's result equals n_steps calls
 * of smrt_step on it alone with the batch's launch shape, bit for bit.
 * Requires an SM scheme, lo_precond = 0 and no reflective side on every
 * problem, and at most 64 problems (else SMRT_E_INVALID_ARG).  Stops after
 * the first step in which a problem fails and returns that status (message
 * in smrt_batch_last_error; strict turns a capped iteration into
 * SMRT_E_NOT_CONVERGED); SMRT_E_DEVICE if a grid-barrier wait of the LO
 * launch exceeds its bound (workgroups not all resident). */
smrt_status smrt_batch_run(smrt_batch *batch, int n_steps, const double *dt, smrt_step_stats *stats,
                           int capture_graph);

/* ------------------------------------------------------------------------
 * Unstructured quadrilateral meshes (the paper's refined meshes have
 * trapezoidal corner cells; Sec. 6).  The lumped bilinear DG sweep of
 * Eq. dgsn_transport on general convex quadrilaterals: at vertex m of a
 * cell the bilinear map's Jacobian J_m gives the lumped weight det(J_m)/4
 * and the basis gradients; each edge's normal times length is split evenly
 * between its two vertices.  Cells are swept per direction in dependency
 * levels, in one launch: a workgroup per (direction, block of 4 groups)
 * walks its direction's levels with a workgroup barrier between them.
 * ------------------------------------------------------------------------ */
typedef struct smrt_qmesh smrt_qmesh;

/* n_vertices points xy[v][2]; n_cells cells[c][4] vertex indices listed
 * counter-clockwise (node n = 4c + l is vertex l of cell c); the quadrature
 * (weights > 0 summing to 4 pi; omega[d][0..1] used); G groups; precision of
 * the sweep.  Boundary edges are numbered in (cell, edge) order, edge e
 * joining vertices e and e+1 (mod 4); boundary node 2k + j is the j-th
 * endpoint of boundary edge k.  Errors: SMRT_E_INVALID_ARG (NULL or empty
 * mesh, index out of range, a cell that is not convex and counter-clockwise,
 * an edge shared by more than two cells, a direction whose upwind
 * dependencies form a cycle), SMRT_E_OUT_OF_MEMORY, SMRT_E_DEVICE.
 * hip_stream: a hipStream_t, or NULL for one owned by the mesh.  Copies
 * everything it needs. */
smrt_status smrt_qmesh_create(int n_vertices, const double *xy, int n_cells, const int32_t *cells,
                              const smrt_quad_desc *quad, int G, smrt_precision precision, void *hip_stream,
                              smrt_qmesh **out);
void smrt_qmesh_destroy(smrt_qmesh *mesh);
const char *smrt_qmesh_last_error(const smrt_qmesh *mesh);
/* Number of boundary nodes and of dependency levels (the most of any direction). */
smrt_status smrt_qmesh_info(const smrt_qmesh *mesh, int *n_boundary_nodes, int *n_levels);
/* One sweep of every (d, g): sig_t[cell][G] (> 0, incl. time absorption),
 * q_iso[node][G], psi_prev[d][g][node] or NULL (zero), inv_c_dt >= 0,
 * inflow[d][g][boundary node] or NULL (vacuum), all host FP64; psi_out
 * [d][g][node] FP64 host; ms_kernel (may be NULL) receives the time of the
 * sweep launches.  Errors: SMRT_E_INVALID_ARG, SMRT_E_DEVICE. */
smrt_status smrt_qmesh_sweep(smrt_qmesh *mesh, const double *sig_t, const double *q_iso, const double *psi_prev,
                             double inv_c_dt, const double *inflow, double *psi_out, double *ms_kernel);
/* Gray angular moments (the moment sums of Sec. 2 over directions and
 * groups) of the intensity left on the device by the last successful
 * smrt_qmesh_sweep on this mesh, in the rectilinear path's 27-row layout:
 * mom_out[27][4 * n_cells] FP64 host, rows 6q..6q+5 = sum over the
 * directions of quadrant q (0: mu > 0 and eta > 0; 1: mu < 0 < eta; 2: both
 * < 0; 3: the rest) and all groups of w f I with f = 1, mu, eta, mu^2,
 * mu eta, eta^2; rows 24..26 = sum of sig w (1, mu, eta) I.  sig[cell][G]
 * (finite, >= 0) host FP64 is the opacity weighting the last three rows.
 * Summed in FP64 on the GPU; ms_kernel (may be NULL) receives the kernel's
 * time.  Errors: SMRT_E_INVALID_ARG (NULL, bad sig, or no sweep yet),
 * SMRT_E_OUT_OF_MEMORY, SMRT_E_DEVICE. */
smrt_status smrt_qmesh_moments(smrt_qmesh *mesh, const double *sig, double *mom_out, double *ms_kernel);

/* ---- Time steps on the mesh: the unaccelerated scheme of Algorithm 1 ----
 * (no low-order solve: each outer iteration sweeps with the emission at the
 * temperature iterate and the time-edge source I^k / (c dt), then solves the
 * pointwise energy balance c_v T/dt + sigma_P a c T^4 = sum_g sigma_g phi_g
 * + c_v T^k / dt; the outer test and caps of smrt_step).  The SM closures are
 * not built on unstructured meshes: their half-range sums are needed for
 * every face normal.
 *
 * Materials: region[n_cells] in [0, n_regions); model 0: sigma0[r][G]
 * tabulated, model 1: sigma_g = sigma0[r] / (nubar_g^3 T^3) clipped to
 * [clip_lo, clip_hi] (nubar_g the geometric mean of the group bounds), T the
 * cell mean of its 4 nodal values, taken once per step at the start-of-step
 * temperature; c_v[r] > 0; nu_edges[G+1] increasing; a, c > 0.  Copied.
 * Setting the materials again discards the state (set it again before a
 * step).  Errors: SMRT_E_INVALID_ARG. */
smrt_status smrt_qmesh_set_materials(smrt_qmesh *mesh, const int32_t *region, int n_regions, int model,
                                     const double *sigma0, double clip_lo, double clip_hi, const double *cv,
                                     const double *nu_edges, double a, double c);
/* State: T[4 n_cells] > 0 at the nodes; psi[d][g][node] the intensity, or
 * NULL for the isotropic equilibrium B_g(T)/4pi.  E = sum_d w_d sum_g I / c
 * follows from psi.  Requires smrt_qmesh_set_materials. */
smrt_status smrt_qmesh_set_state(smrt_qmesh *mesh, const double *T, const double *psi);
/* One backward-Euler step of length dt with the boundary inflow
 * inflow[d][g][NB] (NULL: vacuum) held fixed; opt: scheme must be
 * SMRT_UNACCELERATED and fixup 0 (else SMRT_E_INVALID_ARG); eps_outer,
 * max_outer, fixed_outer, elim_rtol, max_elim, T_floor and strict as for
 * smrt_step.  stats (may be NULL): outer, elim_max, hit_max, t_total_ms.
 * Errors: SMRT_E_NONPHYSICAL (no positive root without a floor, non-finite
 * iterate; the state is left as it was before the step),
 * SMRT_E_NOT_CONVERGED (strict and a cap reached; the state is advanced to
 * the last iterate). */
smrt_status smrt_qmesh_step(smrt_qmesh *mesh, double dt, const double *inflow, const smrt_options *opt,
                            smrt_step_stats *stats);
/* The state after the last step (any pointer may be NULL): T, E [4 n_cells],
 * psi [d][g][node]. */
smrt_status smrt_qmesh_get_state(smrt_qmesh *mesh, double *T, double *E, double *psi);

#ifdef __cplusplus
}
#endif
#endif
