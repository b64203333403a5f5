/*
 * dotsocp.h -- C ABI of the gfx950 (MI355X) solver for dynamic optimal
 * transport on a staggered space-time grid, recast as a linear second-order
 * cone program and solved by the inexact proximal augmented Lagrangian method
 * (Chen, Lin & Zhou, arXiv 2505.05424, Algorithm 2).
 *
 * Every function returns 0 (DOT_OK) on success or a negative dot_status; no
 * C++ exception crosses this boundary. dot_last_error() returns a message for
 * the most recent failure on the calling thread.
 *
 * ---------------------------------------------------------------------------
 * Problem and grids (Sec. 2.2)
 *   D spatial dimensions (1..3); n[0] = n0 time segments, n[1..D] spatial
 *   segments; h_d = 1/n_d. Nodes G^c: (n0+1) x (n1+1) x ... x (nD+1).
 *   Cells G^s_0 (time t+1/2, spatial node x): n0 x (n1+1) x ... (the cones).
 *   G^s_d (d >= 1): time node t, staggered point s+1/2 on axis d.
 *   rho0, rho1: node masses on the spatial nodes (C order, last axis
 *   fastest), non-negative, finite, equal totals (relative mismatch at most
 *   1e-12); they give the boundary vector c of eq. defc. An optional mask
 *   (1 = obstacle) gives the cell weights omega of the weighted problem of
 *   Sec. 5.4.5: omega = 1e-6 on obstacle nodes, 1 elsewhere, time-invariant.
 *   Internally c is divided by h0*h1*...*hD, so the multipliers come out as
 *   density (alpha0 = rho) and momentum density (alpha_d = m_d).
 *
 * Device data layout ("padded box", used by every device pointer below)
 *   A plane is an array of NB = (n0+1)*(n1+1)*...*(nD+1) scalars indexed like
 *   the node grid (time slowest, last spatial axis fastest). A cell-valued
 *   plane (q0, alpha0, one cone component) leaves its time slice n0 unused;
 *   a G^s_d plane (q_d, alpha_d) leaves the slice x_d = n_d unused. Unused
 *   entries must be zero on input and are written as zero.
 *     q, alpha : D+1 consecutive planes (d = 0..D)
 *     beta, z  : K = 4D+2 consecutive planes, component order
 *                [1 - q0 side, (d=1,v=1..4), ..., (d=D,v=1..4), 1 + q0 side]
 *                as in eq. bdd / eq. operBF.
 *   phi, the right-hand side b and the multipliers alpha (which accumulate
 *   small updates every iteration) are always double planes. The bulk state
 *   (q, beta, z and the cone workspace) is double in DOT_FP64 mode and
 *   float in DOT_MIXED mode (dot_plan_info.scalar_bytes); in DOT_MIXED the
 *   cosine transforms run in float on the correction of phi (defect
 *   correction: A^*A dphi = b - A^*A phi, phi += dphi, in double), while the
 *   cone projection, A phi and every reduction stay in double.
 *
 * Ownership: the caller owns every buffer it passes; the library keeps no
 * pointer to caller memory after a call returns. A dot_plan owns only small
 * constant tables on its device (transform matrices, eigenvalues, weights).
 * Streams are hipStream_t passed as void*; NULL means the default stream.
 * All step functions are asynchronous on that stream.
 */
#ifndef DOTSOCP_H
#define DOTSOCP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DOT_OK = 0,
  DOT_EINVAL = -1,   /* invalid argument or problem data */
  DOT_ENOMEM = -2,   /* a device or host allocation failed */
  DOT_EDEVICE = -3,  /* a HIP runtime call failed */
  DOT_EBUSY = -4     /* a serving request can never fit the HBM budget */
} dot_status;

typedef enum { DOT_FP64 = 0, DOT_MIXED = 1 } dot_precision;

typedef enum {
  DOT_RUNNING = -1,
  DOT_CONVERGED = 0, /* eta_dot <= tol at a residual check */
  DOT_MAXITER = 1,   /* iteration cap reached */
  DOT_TIMEOUT = 2,   /* time_limit_s ran out (the state can be continued) */
  DOT_DIVERGED = 3   /* a residual became NaN or Inf */
} dot_term;

typedef struct {
  int32_t D;              /* 1..3 */
  int32_t n[4];           /* n[0] = n0 >= 1 time segments; n[1..D] >= 1 */
  const double* rho0;     /* host, prod_d (n_d+1) node masses, >= 0 */
  const double* rho1;     /* host, same shape and total mass */
  const uint8_t* mask;    /* host, optional (NULL): 1 = obstacle */
  double tol;             /* stop when eta_dot <= tol; < 0: never stop */
  int32_t max_iter;       /* iteration cap (> 0) */
  int32_t precision;      /* dot_precision */
  double tau;             /* dual step in (0, 2); 0 selects 1.9 */
  double sigma0;          /* initial penalty; 0 selects 30 */
  int32_t check_every;    /* residual-check cadence; 0 selects 5 */
  int32_t adapt_sigma;    /* 1: sigma rule of Sec. 5.3 on the growing schedule */
  int32_t sigma_gap0;     /* first sigma decision after this many iterations; 0 selects 10 */
  double sigma_growth;    /* gap growth g' = floor(growth*g) + check_every, rounded down
                             to a multiple of check_every; 0 selects 1.2 */
  double time_limit_s;    /* wall-clock budget in seconds (0: none). dot_run / dot_batch_run:
                             per call; when it runs out the call returns at its next poll of
                             the control blocks (every 40 iterations) with term DOT_TIMEOUT
                             and the state resumable. Serving: from the request's admission
                             (on its target level); the request is retired at the next step
                             with DOT_TIMEOUT and its iterate so far */
} dot_problem;

typedef struct {
  double objective;       /* -<c, phi> in unscaled units (about W2^2 / 2) */
  double dual_objective;  /* 1/2 sum_d sum_{r_d>0} m_d^2 / r_d (unscaled) */
  double eta_dot, eta_p, eta_d, eta_c, eta_p_soc, eta_d_soc;
  double sigma;           /* penalty after the last check */
  int32_t iters;          /* PALM iterations done */
  int32_t term;           /* dot_term */
  int32_t checks;         /* residual checks done */
  int32_t sigma_changes;  /* sigma decisions that changed sigma */
} dot_result;

typedef struct {
  int32_t D, K;
  int32_t n[4];
  int64_t nb;             /* scalars per plane */
  int32_t scalar_bytes;   /* 8 (FP64) or 4 (MIXED bulk) */
  int32_t n_planes;       /* bulk-type planes in the state buffer (q, q_new, beta, W) */
  size_t state_bytes;     /* bytes the caller must provide for a state buffer */
  /* byte offsets inside a state buffer: phi (FP64 plane), transform scratch
   * (mixed precision only), q, q_new (bulk type), alpha (double), beta, W (4D planes of the
   * bulk type, then one double plane of z-step workspace) */
  uint64_t off_phi, off_scratch, off_q, off_qn, off_alpha, off_beta, off_w;
} dot_plan_info;

typedef struct dot_plan dot_plan;

const char* dot_last_error(void);

/* Validate p (mass balance, sizes, finite data), build c, omega, the cosine
 * transform tables and eigenvalues of A^*A (Sec. 4, phi-step of Algorithm 2) on the
 * current HIP device. The plan copies everything it needs from p. DOT_EINVAL
 * if a transformed axis (every axis but a last one of >= 257 nodes) exceeds
 * what one transform tile holds (about 1100 nodes in FP64, 2200 mixed). */
int dot_plan_create(const dot_problem* p, dot_plan** out);
void dot_plan_destroy(dot_plan* plan);
int dot_plan_get_info(const dot_plan* plan, dot_plan_info* out);

/* Initial point of Algorithm 1: q = alpha = beta = 0 (0 lies in Q), sigma =
 * sigma0, counters cleared. `state` is a device buffer of info.state_bytes. */
int dot_state_reset(dot_plan* plan, void* state, void* stream);

/* Run PALM iterations of Algorithm 2 on `state` until eta_dot <= tol at a
 * residual check, or `max_iters` more iterations, on `stream`; blocks until
 * done and fills *res (may be NULL). Residual checks and the sigma rule run on
 * the device every check_every iterations. */
int dot_run(dot_plan* plan, void* state, int32_t max_iters, void* stream, dot_result* res);

/* Copy rho = alpha0 (n0 x prod(n_d+1), density at half-times) and the D
 * momentum blocks m_d = alpha_d (exact G^s_d shapes, concatenated) from a
 * state buffer into host arrays (either may be NULL). */
int dot_extract(dot_plan* plan, const void* state, double* rho_out, double* m_out, void* stream);

/* ---- step-level entry points (one row of the hot path each) ------------ */

/* a3: b = A^*(q - alpha/sigma) - c/sigma (right-hand side of the phi-step of
 * Algorithm 2), node plane b. */
int dot_step_divergence(dot_plan* plan, const void* q, const void* alpha, double sigma,
                        void* b, void* stream);
/* a4: phi = (A^*A)^+ b in place on the node plane (phi-step of Algorithm 2): forward
 * DCT-II on every axis, divide by the eigenvalues, zero mode set to 0 (phi in
 * rge A^*), inverse transform. A last axis of 257 or more nodes is not
 * transformed: after the other axes' transforms each of its lines is a
 * tridiagonal system (eigenvalue sum of the other axes + path-graph Laplacian
 * / h^2), solved by elimination with the recurrences in FP64 registers; same
 * linear system, same phi up to rounding (forward error within the condition
 * number of the line systems times the FP64 unit, which grows with the square
 * of the axis length). In DOT_MIXED the transforms work on an FP32 plane; a
 * line of up to 576 nodes is eliminated with its values staged in FP64 (LDS
 * and registers) between one FP32 load and one FP32 store, while the
 * one-lane elimination of longer lines keeps its intermediate d' between the
 * forward and backward sweep in the plane's type (the c' checkpoints are
 * FP64), i.e. the FP32 rounding of the other transform passes. Such
 * an axis has no transform-tile limit (every axis stays within the 4096
 * segments dot_plan_create accepts); the other axes must fit a tile. */
int dot_step_poisson(dot_plan* plan, void* b_to_phi, void* stream);
/* a3 + a4 as the iteration runs them (right-hand side sweep, then the
 * transform passes): phi from (q, alpha, sigma). */
int dot_step_rhs_poisson(dot_plan* plan, const void* q, const void* alpha, double sigma,
                         void* phi, void* stream);
/* a1 + a2: z = Pi_Q(B_omega F q + d - beta/sigma) (z-step of Algorithm 2; eq. app-proj
 * per cell, eq. fdetails for the gather), K planes. */
int dot_step_cone(dot_plan* plan, const void* q, const void* beta, double sigma,
                  void* z, void* stream);
/* a5: q_new, alpha, beta updates of Algorithm 2 (q-step and both
 * multiplier steps) from phi and the old
 * (q, alpha, beta); alpha and beta are updated in place, q_new written to
 * q_out; w_scratch is workspace for the z-step: 4D planes of the bulk type
 * followed by one double plane (nb * (4D * scalar_bytes + 8) bytes). */
int dot_step_update(dot_plan* plan, const void* phi, const void* q, void* alpha, void* beta,
                    double sigma, double tau, void* q_out, void* w_scratch, void* stream);
/* a6: the relative KKT residuals of Sec. 5.3 at (phi, z, q, alpha, beta),
 * the objective and the dual objective; blocks and fills *res (iters and
 * term are left 0). */
int dot_step_residuals(dot_plan* plan, const void* phi, const void* z, const void* q,
                       const void* alpha, const void* beta, dot_result* res, void* stream);

/* ---- residuals without device allocation --------------------------------- */
/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc. Computes what
 * dot_step_residuals computes (the relative KKT residuals of Sec. 5.3, the
 * objective and the dual objective at (phi, z, q, alpha, beta); same kernels,
 * same summation order, so bitwise the same result) and calls no hipMalloc,
 * hipFree or other allocating routine: the control block and the
 * per-workgroup partial sums go to a fixed device array of
 * DOT_NOALLOC_SCRATCH_BYTES that the library holds on each GPU it runs on
 * until the process ends, instead of the plan's buffers. A plan needs 768
 * bytes for the control block plus 160 bytes per workgroup of its residual
 * sweep (about 9,700 workgroups for 3D 32x64^3, 37,000 for 2D 32x1024^2) and
 * 10,240 bytes for the first stage of their reduction;
 * beyond the array's size the call returns DOT_EINVAL before any device work.
 * The current device must be the plan's (DOT_EINVAL otherwise). Every call on
 * one GPU shares that GPU's array and leaves the last call's contents in it;
 * calls that overlap on one GPU (other streams or host threads) race. Blocks
 * and fills *res (iters and term are left 0 / DOT_RUNNING). */
#define DOT_NOALLOC_SCRATCH_BYTES (8u << 20)
int dot_step_residuals_noalloc(dot_plan* plan, const void* phi, const void* z, const void* q,
                               const void* alpha, const void* beta, dot_result* res, void* stream);

/* ---- measurement hook ---------------------------------------------------- */
/* Kernel classes of one iteration, for dot_profile_select. */
typedef enum {
  DOT_K_DCT_FIRST = 0, /* time-axis forward pass */
  DOT_K_DCT_MID = 1,   /* forward passes on the middle spatial axes */
  DOT_K_DCT_LAST = 2,  /* last axis: forward, 1/Lambda, inverse (or its tridiagonal elimination) */
  DOT_K_DCT_INV = 3,   /* inverse passes on the other axes */
  DOT_K_CONE = 4,      /* cone gather + projection (z-step) into the weighted w planes */
  DOT_K_QD = 5,        /* q-step and alpha update (q0 and q_d) */
  DOT_K_BETA = 6,      /* beta update */
  DOT_K_RESID = 7,     /* residual partial sums (checks only) */
  DOT_K_FINAL = 8,     /* residual finalize + sigma rule (checks only) */
  DOT_K_RHS = 9,       /* right-hand side A^*(q - alpha/sigma) - c/sigma (mixed: its defect) */
  DOT_K_NONE = -1
} dot_kernel_class;

/* Record HIP events around every launch of one kernel class inside dot_run
 * on its stream (DOT_K_NONE switches recording off); dot_profile_read returns
 * the summed event time in ms and the number of launches since the last read
 * and clears them. While a class is recorded, graphs are off and every class
 * runs as its own launch (otherwise an iteration without a residual check
 * computes the next iteration's z-step and right-hand side inside its beta
 * launch, and large instances run the z-step beside the phi-step). */
int dot_profile_select(dot_plan* plan, int32_t kernel_class);
int dot_profile_read(dot_plan* plan, double* total_ms, int64_t* launches);

/* ---- batches: many instances, one launch per kernel of an iteration ------ */
/* A batch holds `count` problems with the same D, precision and check
 * cadence but any grid sizes, masks and data. Every kernel of an iteration is
 * launched once for all instances; per-instance descriptors (geometry, state
 * pointers, tables) and block maps route each workgroup to its instance. Each
 * instance keeps its own sigma, residuals and stop flag on the device, stops
 * on its own, and gives bitwise the same iterates as a solve of that problem
 * alone (same kernels, fixed-order reductions). The caller provides one device
 * workspace of dot_batch_workspace_bytes. */
typedef struct dot_batch dot_batch;
int dot_batch_create(const dot_problem* probs, int32_t count, dot_batch** out);
void dot_batch_destroy(dot_batch* batch);
size_t dot_batch_workspace_bytes(const dot_batch* batch);
int32_t dot_batch_size(const dot_batch* batch);
/* zero state, sigma0 and counters for every instance */
int dot_batch_reset(dot_batch* batch, void* workspace, void* stream);
/* up to max_iters iterations of all instances in lockstep (stopped instances
 * do no work); blocks; fills results[count] (may be NULL). Compaction: at the
 * start of the call and at each poll of the control blocks (every 40
 * iterations) the launches are laid out anew over the instances still running
 * once the stopped ones hold at least 1/8 of the workgroups of a node sweep,
 * so stopped instances stop taking dispatch slots (their descriptors and
 * states stay; results are unchanged). Time budgets
 * (dot_problem.time_limit_s): the call returns at the first poll after the
 * smallest nonzero budget among the instances has run out, unless it has done
 * max_iters iterations by then. On such an early return an unfinished
 * instance whose own budget has run out reports DOT_TIMEOUT; the other
 * unfinished instances (no budget, or one not yet spent) report DOT_RUNNING.
 * Every state is resumable by another dot_batch_run. */
int dot_batch_run(dot_batch* batch, void* workspace, int32_t max_iters, void* stream, dot_result* results);
/* Instances that have workgroups in the batch's launches (all after
 * dot_batch_create and dot_batch_reset; fewer after a run that compacted the
 * layout); -1 for a null batch. */
int32_t dot_batch_laid_out(const dot_batch* batch);
/* rho / m of instance `index`, as dot_extract */
int dot_batch_extract(dot_batch* batch, const void* workspace, int32_t index, double* rho_out, double* m_out,
                      void* stream);
int dot_batch_profile_select(dot_batch* batch, int32_t kernel_class);
int dot_batch_profile_read(dot_batch* batch, double* total_ms, int64_t* launches);

/* Replay captured HIP graphs (blocks of 10 iterations, and the 40 iterations
 * between two polls of the control blocks) inside dot_run / dot_batch_run
 * and the serving steps (default on; off runs the same launches one by one;
 * results are bitwise identical). Graphs are not used while a kernel class
 * is being timed. A capture that fails leaves its block to plain launches of
 * the same kernels; after two failures a run call stops capturing. Either
 * call drops the graphs captured so far. */
int dot_plan_set_graphs(dot_plan* plan, int32_t enable);
int dot_batch_set_graphs(dot_batch* batch, int32_t enable);
/* Testing the fallback above: the next `count` graph captures in this
 * process fail before they start (0 clears; DOT_EINVAL if negative). */
int dot_test_fail_captures(int32_t count);

/* ---- transform schedules and their autotuner ----------------------------- */
/* The cosine-transform passes of the phi-step (Sec. 4, the Poisson solve of
 * Algorithm 2) run one workgroup per tile of cw lines of an axis, with `waves`
 * 64-lane wavefronts per workgroup. By default both come from a rule on the
 * launch's line count. A schedule changes no computed value: every line's
 * products run in one wavefront in a fixed order, so results are bitwise
 * those of any other schedule (and a batch member still equals its solve
 * alone). On a last axis that every instance of the launch solves by
 * tridiagonal elimination (>= 257 nodes) cw is the number of lines of each
 * 256-thread workgroup: 4, 8, 16, 32 or 64 (4 and 8 only when no line is
 * longer than 576 nodes), by default the lines one round of the partitioned
 * solve takes (8 for lines of up to 288 nodes, 4 up to 576; 64 when some
 * line is longer); waves do not apply. */
typedef struct {
  int32_t cw[4];       /* lines per tile, axes 0..D: 16, 32 or 64, also 4 or 8 on an eliminated last
                          axis (set calls: 0 keeps the rule's) */
  int32_t waves[4];    /* wavefronts per workgroup, 1..16, enough for the axis's work items
                          (set calls: 0 keeps the rule's for that tile width) */
  int32_t tuned;       /* out: 1 when the schedule was chosen by an autotune call */
  int32_t candidates;  /* out: schedules the autotune call timed */
  double us;           /* out (autotune): one transform sequence (all passes of one phi-step), us */
  double us_rule;      /* out (autotune): the same with the rule's schedule */
} dot_schedule;

/* Install a schedule (NULL: the rule's) for later runs; DOT_EINVAL when an
 * axis's tile does not fit the LDS of some instance or the waves cannot hold
 * its work items (the schedule in use is then kept). Captured graphs are
 * dropped and re-captured on the next run. The batch call waits until the
 * device is idle before it releases the previous block maps. None of the
 * schedule calls may overlap a run of the same plan or batch, or be made
 * inside a graph capture. */
int dot_plan_set_schedule(dot_plan* plan, const dot_schedule* schedule);
int dot_batch_set_schedule(dot_batch* batch, const dot_schedule* schedule);
/* The schedule in use (the rule's values written out when none is set). */
int dot_plan_get_schedule(const dot_plan* plan, dot_schedule* out);
int dot_batch_get_schedule(const dot_batch* batch, dot_schedule* out);
/* Autotuner: times the transform sequence with HIP events on `stream` for
 * every candidate schedule (each tile width the axis fits; per width the
 * fewest waves that hold its work items, 4, 8, 16, one per item and the
 * rule's), one axis at a time with the others at their best so far, and
 * installs the fastest (the rule's unless a measured schedule beats it).
 * The state / workspace is overwritten and left as after dot_state_reset /
 * dot_batch_reset. Blocks; fills *out (may be NULL). */
int dot_plan_autotune(dot_plan* plan, void* state, void* stream, dot_schedule* out);
int dot_batch_autotune(dot_batch* batch, void* workspace, void* stream, dot_schedule* out);

/* One-shot, blocking: allocate, solve, copy rho/m out (either may be NULL),
 * free. rho_out: n0*prod(n_d+1); m_out: sum_d |G^s_d| doubles. */
int dot_solve(const dot_problem* p, double* rho_out, double* m_out, dot_result* res);

/* ---- multilevel initialisation ------------------------------------------ */
/* The multilevel strategy of the paper (implementation details of Sec. 5.3,
 * experiments of Sec. 5.4): solve on grids with n_d / 2^v segments,
 * v = L..1, and start each finer level from the linear interpolation of the
 * coarser solution; level v is solved to max{tol * 10^-v, 1e-6}. */

/* Data of the next coarser grid (n_d / 2 segments on every axis; every n_d
 * must be even and >= 2). Host arrays: node masses are restricted with the
 * transpose of linear interpolation (fine node 2i gives all its mass to coarse
 * node i, fine node 2i+1 half to each of i and i+1), which keeps the total
 * mass; with a mask, coarse node i is an obstacle node when fine node 2i is,
 * carries no mass, and each density is renormalised to its total. Outputs
 * hold prod_d (n_d/2 + 1) entries (mask_out only if mask is given). */
int dot_coarsen_data(int32_t D, const int32_t* n, const double* rho0, const double* rho1, const uint8_t* mask,
                     double* rho0_out, double* rho1_out, uint8_t* mask_out);
/* Initial point of the finer level: q, alpha and beta of fine_state become the
 * tensor-product linear interpolation of those of coarse_state (positions of
 * each staggered set in physical coordinates, constant beyond the outermost
 * coarse positions), phi, z-weights and q_new are zeroed, sigma carries over
 * and the iteration counter and sigma schedule restart. The plans need the
 * same D and precision and fine n[d] = 2 * coarse n[d]. Blocks. */
int dot_prolong(const dot_plan* coarse, const void* coarse_state, dot_plan* fine, void* fine_state, void* stream);

/* ---- checkpoint / warm start --------------------------------------------- */
/* The iterate of Algorithm 2 (q, alpha, beta and sigma) in and out of a state
 * (restarting from the latest iterate, as the paper does when sigma changes,
 * Sec. 5.3). Host FP64 arrays in the padded-box layout of dot_plan_info: nb
 * scalars per plane in node order (time slowest, last spatial axis fastest);
 * q and alpha hold D+1 planes (q0 / alpha0 on cells: time slices t < n0;
 * q_d / alpha_d on G^s_d: x_d < n_d), beta K planes (cells). */
/* Copies out the newest iterate and sigma (any output may be NULL); positions
 * outside a plane's set are zero. Mixed precision: q and beta widened exactly
 * from FP32. Blocks. */
int dot_state_export(const dot_plan* plan, const void* state, double* q, double* alpha, double* beta, double* sigma,
                     void* stream);
/* Starts `state` from a given iterate: zero state, then q, alpha, beta (values
 * outside a plane's set are ignored; mixed precision rounds q and beta to
 * FP32) and sigma (> 0); phi and the z-weights start at zero and the
 * iteration and check counters and the sigma schedule start anew, as for a
 * new solve. DOT_EINVAL for a non-finite value or sigma. Blocks. */
int dot_state_import(dot_plan* plan, void* state, const double* q, const double* alpha, const double* beta,
                     double sigma, void* stream);

/* ---- sigma history -------------------------------------------------------- */
/* The penalty changes of the sigma rule (Sec. 5.3) made so far in `state`:
 * the new sigma and the iteration count of the check that made each change,
 * oldest first; the control block keeps the last 32, and at most `cap` of
 * them (the newest) are written. *count receives the number of changes
 * overall (equal to dot_result.sigma_changes). Outputs may be NULL. Blocks. */
int dot_sigma_history(const dot_plan* plan, const void* state, double* sigma, int32_t* at_iter, int32_t cap,
                      int32_t* count, void* stream);
int dot_batch_sigma_history(const dot_batch* batch, const void* workspace, int32_t index, double* sigma,
                            int32_t* at_iter, int32_t cap, int32_t* count, void* stream);

/* ---- finishing a mixed-precision solve in FP64 -------------------------- */
/* Continue the iterate of Algorithm 2 held in `mixed_state` (a state of
 * `mixed_plan`, DOT_MIXED) in `fp64_state` (a state of `fp64_plan`, DOT_FP64,
 * made from the same problem: same grid, data and check cadence; grid and
 * cadence are checked). phi and alpha are copied (FP64 in both layouts), q,
 * q_new and beta widened exactly from FP32, the z-weight planes cleared (they
 * carry values only inside an iteration); sigma, the residuals of the last
 * check, the iteration and check counters and the sigma schedule carry over,
 * tau / tol / the sigma-rule switch come from fp64_plan, and the stop flag is
 * cleared. dot_run on fp64_plan then continues where the mixed run stopped.
 * For mixed runs that level off above their tolerance at the FP32 storage
 * floor. mixed_state is not modified. Blocks. */
int dot_state_promote(const dot_plan* mixed_plan, const void* mixed_state, dot_plan* fp64_plan, void* fp64_state,
                      void* stream);
/* The same for instance `index` of a DOT_MIXED batch (its state and control
 * block in the batch workspace `workspace`): fp64_plan must be made from that
 * instance's problem in DOT_FP64. The batch is not modified. */
int dot_batch_promote(const dot_batch* batch, const void* workspace, int32_t index, dot_plan* fp64_plan,
                      void* fp64_state, void* stream);
/* The same into member `slot` of a DOT_FP64 batch (`fp64_batch`, workspace
 * `fp64_workspace`), whose problem at that slot must be instance `index`'s
 * problem: its state and control block are overwritten, so that
 * dot_batch_run on the FP64 batch continues every promoted member together
 * (one launch per kernel, each member bitwise as dot_batch_promote +
 * dot_run). Members of a batch iterate in lockstep, so the FP64 batch takes
 * the mixed batch's iteration count: DOT_EINVAL if it has already run to
 * another count (promote after dot_batch_reset, all from one mixed batch and
 * iteration). Members not promoted keep their state (after a reset: zero, as
 * a fresh solve). Blocks. */
int dot_batch_promote_member(const dot_batch* batch, const void* workspace, int32_t index, dot_batch* fp64_batch,
                             void* fp64_workspace, int32_t slot, void* stream);
/* One-shot multilevel solve with `levels` coarser grids (0 = plain solve):
 * allocates, solves level by level on the default stream, copies rho / m of
 * the target grid (as dot_solve) and frees. res: the target level;
 * level_results (may be NULL): levels + 1 entries, coarsest first. max_iter
 * caps every level. */
int dot_solve_multilevel(const dot_problem* p, int32_t levels, double* rho_out, double* m_out, dot_result* res,
                         dot_result* level_results);

/* ---- serving: continuous batching under an HBM budget --------------------- */
/* A serving context holds one device arena of hbm_budget_bytes and up to
 * max_slots running instances of one D and precision. Requests queue in
 * arrival order. dot_ctx_step admits queued requests while a slot and arena
 * space exist (first fit; the queue head waits for space, later requests do
 * not overtake it), runs `iters` iterations of every running instance (one
 * launch per kernel over all of them, Algorithm 2 as in dot_batch_run), then
 * retires every instance that converged, diverged or reached its max_iter:
 * its rho / m and result are copied to host memory inside the context and its
 * arena block and slot are freed for the next admissions. Admissions happen
 * at multiples of 10 iterations of the context's counter, so each request
 * follows exactly the iterates of a solve of that problem alone (dot_run with
 * the same settings): same result fields, bitwise. Requests need the default
 * check cadence (5) and a max_iter that is a multiple of 5. Every dot_ctx_*
 * call takes the context's lock and makes the context's device current for
 * its duration (the caller's current device is restored), so several host
 * threads may share one context; a dot_ctx_step holds the lock until its
 * iterations are done. dot_last_error() keeps the calling thread's last
 * failure, dot_ctx_last_error() the context's. */
typedef struct dot_ctx dot_ctx;
typedef enum { DOT_REQ_QUEUED = 0, DOT_REQ_RUNNING = 1, DOT_REQ_DONE = 2 } dot_req_status;
/* Device bytes one instance of p's D, n and precision takes in the arena
 * (state, control block and reduction partials); 0 for an invalid D. Pure host
 * arithmetic; the rho/mask pointers of p are not read. */
size_t dot_footprint_bytes(const dot_problem* p);
/* Reserves the arena on HIP device `device` (-1: the current device) for
 * requests of D spatial dimensions and one precision, with at most max_slots
 * running at a time (1..4096). DOT_EINVAL for a device index outside the
 * devices present or bad arguments; DOT_ENOMEM if the device cannot hold the
 * budget. Later calls on the context run on that device whatever the caller's
 * current device, on the stream they are given. */
int dot_ctx_create(int32_t device, int32_t D, int32_t precision, size_t hbm_budget_bytes, int32_t max_slots,
                   dot_ctx** out);
/* Frees the arena and every request, finished or not. */
void dot_ctx_destroy(dot_ctx* ctx);
/* Validates p (as dot_plan_create), builds its constant tables and queues it;
 * *ticket identifies it until dot_ctx_fetch. DOT_EBUSY if its footprint
 * exceeds the whole budget; DOT_EINVAL if D / precision differ from the
 * context's. The host arrays of p are copied before return. */
int dot_ctx_submit(dot_ctx* ctx, const dot_problem* p, uint64_t* ticket);
/* As dot_ctx_submit, for the multilevel solve of dot_solve_multilevel (the
 * multilevel initialisation of Sec. 5.3): the coarse problems are built at
 * submission (levels in 0..8; 0 is dot_ctx_submit), the request reserves the
 * states of all levels in one arena block and iterates the coarsest level
 * first; when a level stops (converged, diverged or at max_iter) its iterate
 * is interpolated into the next finer level's state, sigma carried, and that
 * level starts at the next step. Only the target level retires; its rho / m
 * and result are what dot_ctx_fetch returns, bitwise those of
 * dot_solve_multilevel with the same settings. */
int dot_ctx_submit_ml(dot_ctx* ctx, const dot_problem* p, int32_t levels, uint64_t* ticket);
/* Admit, run iters (a multiple of 10) iterations, retire; blocks until the
 * work is done. Optional outputs: running and queued counts after the step.
 * With nothing running, only admission happens. */
int dot_ctx_step(dot_ctx* ctx, int32_t iters, void* stream, int32_t* n_active, int32_t* n_queued);
/* *status = dot_req_status of the request. */
int dot_ctx_poll(dot_ctx* ctx, uint64_t ticket, int32_t* status);
/* Copies a finished request's rho / m (host, shapes as dot_solve; either may
 * be NULL) and result, then forgets the ticket. DOT_EINVAL if not finished. */
int dot_ctx_fetch(dot_ctx* ctx, uint64_t ticket, double* rho_out, double* m_out, dot_result* res);
/* Free arena bytes and the counts of admitted and retired requests. */
int dot_ctx_stats(const dot_ctx* ctx, size_t* free_bytes, int64_t* admitted, int64_t* retired);
/* Checkpoint of a running request (restart from the latest iterate, Sec. 5.3,
 * here without losing any state), or of a finished one kept at its iteration
 * cap (dot_ctx_keep_capped, before its fetch): between two dot_ctx_step calls, copies the
 * whole device state of the request's current level -- every plane (phi, q,
 * q_new, alpha, beta and the workspaces) and its control block (sigma,
 * counters, sigma schedule, last residuals, iteration cap) -- with a header
 * naming D, precision, grids and level into the host buffer `buf` of `cap`
 * bytes. *bytes receives the size needed; with buf NULL only the size is
 * reported. The request keeps running in this context. DOT_EINVAL for an
 * unknown ticket, a queued request, a finished one without a kept
 * checkpoint, or cap too small. Blocks on `stream`. */
int dot_ctx_export(dot_ctx* ctx, uint64_t ticket, void* buf, size_t cap, size_t* bytes, void* stream);
/* Queues a request that resumes from a checkpoint of dot_ctx_export (made by
 * this or another context with the same D and precision): p and levels must
 * be those of the exported request (grids and layout are checked against the
 * header); the host arrays of p are copied before return. At admission its
 * state and control block are those of the checkpoint, so it continues the
 * exported iterate exactly: it finishes with bitwise the result the exported
 * request would have reached without interruption. The request runs to
 * p->max_iter: a checkpoint of a request that stopped at a smaller cap
 * (dot_ctx_keep_capped) continues from there. A mixed-precision checkpoint
 * imported into an FP64 context is promoted as by dot_state_promote (phi and
 * alpha copied, q, q_new and beta widened exactly, sigma, counters and sigma
 * schedule kept), so the request continues that iterate in FP64. The
 * checkpoint's iteration count must be a multiple of 10 (every export between
 * steps, and a cap that is a multiple of 10, give one). The time budget of p
 * restarts at the new admission. DOT_EINVAL on any mismatch, as
 * dot_ctx_submit otherwise. */
int dot_ctx_import(dot_ctx* ctx, const dot_problem* p, int32_t levels, const void* buf, size_t bytes,
                   uint64_t* ticket);
/* With keep != 0, a request of this context that stops at its max_iter
 * without converging keeps a checkpoint of its final state (the layout of
 * dot_ctx_export) in host memory until dot_ctx_fetch: dot_ctx_export then
 * returns it for the finished request, so that it can continue elsewhere --
 * typically a mixed-precision request whose FP32 state levels off above its
 * tolerance, continued in an FP64 context (see dot_ctx_import). Off by
 * default (a kept checkpoint holds the whole state). */
int dot_ctx_keep_capped(dot_ctx* ctx, int32_t keep);
/* Message of the last failed call on this context ("" if none). */
const char* dot_ctx_last_error(const dot_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* DOTSOCP_H */
