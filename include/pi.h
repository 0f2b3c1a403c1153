/*
 * pi.h -- C interface of libpi, an MI355X (gfx950) solver for matrix-based
 * omnidirectional pressure integration (Zigunov & Charonko, arXiv 2311.16935).
 *
 * Problem (Section "The Matrix-based Omnidirectional Integration Method"):
 * given a pressure-gradient field f on a uniform rectangular 2-D or 3-D grid
 * of cells, some of which hold no data, find the pressure P (up to one
 * constant per connected group of data cells) by iterating Eq. MatrixEquation
 *     [W^{n+1}] {P^{n+1}} = [W^n] {P^n} + {S}
 * from {P^0} (Algorithm 1) until the momentum residual of
 * Eq. ResidualMomentum falls to a threshold.  The weights come from the ray
 * counters of Eqs. AEnp1, AEn, ANnp1, ANn, Acn (2-D) and their 3-D analogues;
 * {S} is the source sum of Eq. ExplicitEqn_FaceCrossing.
 *
 * Conventions shared by every call:
 *  - Grid sizes are (nx, ny[, nz]); arrays are dense, x fastest:
 *    cell (x, y, z) lives at x + nx * (y + ny * z).
 *  - Directions: E = +x, W = -x, N = +y, S = -y, F = +z, B = -z.
 *  - The mask is one byte per cell, 1 = data present, 0 = missing; cells
 *    outside the grid count as missing.
 *  - "Device pointer" means memory from hipMalloc (or a torch CUDA tensor) on
 *    the current HIP device; the library never frees caller memory.
 *  - Precision: with PI_FP32 the gradients and P are float; the operator
 *    apply and the inner Krylov updates run in float, while P is carried in
 *    double internally and every dot product, norm and the gauge are
 *    accumulated in double.  With PI_FP64 everything is double.
 *  - Every call returns a pi_status; no C++ exception crosses the interface.
 *    Calls on one plan are not thread-safe; distinct plans are independent.
 *  - stream is a hipStream_t passed as void* (NULL = the default stream).
 *    Work is enqueued asynchronously unless stated otherwise.
 */
#ifndef PI_H
#define PI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum pi_status {
  PI_OK = 0,
  PI_ERR_INVALID_ARG = 1,   /* a size, spacing, pointer or flag is invalid     */
  PI_ERR_OOM = 2,           /* device or host allocation failed                */
  PI_ERR_NONFINITE = 3,     /* a data cell holds a NaN or infinite gradient    */
  PI_ERR_NOT_CONVERGED = 4, /* max_iter outer steps without reaching tol       */
  PI_ERR_DIVERGED = 5,      /* the residual became non-finite                  */
  PI_ERR_DEVICE = 6,        /* a HIP runtime call failed                       */
  PI_ERR_TOO_LARGE = 7      /* beyond pi_solve_batched_noalloc's fixed scratch */
} pi_status;

typedef struct pi_plan_s *pi_plan_t;

/* pi_plan flags */
#define PI_FP32 0x0u
#define PI_FP64 0x1u
#define PI_INNER_CG 0x0u        /* conjugate gradient, as in the paper's GPU code */
#define PI_INNER_BICGSTAB 0x2u  /* stabilised BiCG, safe for the nonsymmetric M  */
/*
 * Variant, not the paper's iteration: solve the fixed point of Eq.
 * MatrixEquation, ([W^{n+1}] - [W^n]) P = S, directly -- CG on that
 * symmetric operator for the inner correction instead of [W^{n+1}], so the
 * boundary rows are no longer lagged by one outer step.  Same FP64 outer
 * residual, same stopping test (Eq. ResidualMomentum) and same converged
 * field; far fewer passes over the grid.  CG only (not with BiCGStab).
 */
#define PI_FIXED_POINT_CG 0x4u
/*
 * The cell-centred scheme (Section "Method Concept"), 2-D only: a ray's path
 * is the cells whose centres lie nearest to it, one per column for rays less
 * steep than the cell diagonal, one per row otherwise, so a cell takes rays
 * from its 8 face and diagonal neighbours and the pressure is carried from
 * centre to centre with the trapezoid rule (Eq. ExplicitEqn_FaceCrossing
 * with the diagonal directions j).  The weights are the measures of those
 * rays over all angles and offsets: for an interior cell, with D = |(dx,
 * dy)| and A_tot = 4 D, 2 (D - dx) from each x neighbour, 2 (D - dy) from
 * each y neighbour and dx + dy - D from each diagonal one.  At boundaries a
 * ray starts at the first data cell of its path, as in the face-crossing
 * scheme: its weight moves to [W^n] when the cell before the neighbour holds
 * no data, to w_C^n when the neighbour holds none.  The paper gives this
 * scheme's boundary weights only in supplementary material; these follow
 * from the same definition.  Connected groups (gauge) count diagonal
 * neighbours.  Not with PI_INNER_BICGSTAB.
 */
#define PI_CELL_CENTERED 0x8u

/* pi_solve flags */
#define PI_WARM_START 0x1u      /* P holds P^0 on entry (else P^0 = 0)            */
#define PI_ASYNC 0x2u           /* enqueue the whole solve on the stream; see below */

/* operators for pi_apply */
#define PI_OP_M 0  /* [W^{n+1}] = I - W^{n+1}                                    */
#define PI_OP_N 1  /* [W^n] = W^n (diagonal w_C^n)                               */
#define PI_OP_L 2  /* [W^{n+1}] - [W^n], whose residual Eq. ResidualMomentum uses */

typedef struct pi_info {
  int64_t outer_iters;       /* solves of Eq. MatrixEquation performed          */
  int64_t inner_iters_total; /* inner Krylov iterations over all outer steps    */
  double eps_R;              /* Eq. ResidualMomentum at the returned P          */
  double eps_P;              /* Eq. ResidualPressure of the last outer step     */
  double ms;                 /* wall time of the call, host clock, milliseconds */
  int32_t status;            /* pi_status of this instance                      */
  int32_t components;        /* connected groups of data cells                  */
  int32_t worklist_rebuilds; /* batched calls: times the work list was shrunk
                                to the unfinished instances (0 for pi_solve)   */
  int32_t reserved;
} pi_info;

/*
 * pi_plan -- analyse a grid once: ray-count constants (Eq. cxx2D in 2-D;
 * Eqs. FarFaceEquation and IAc..ICc by quadrature in 3-D, or the closed forms
 * of Eqs. ConstantFarFace / ConstantNearFaces when dx = dy = dz), the packed
 * per-cell counter codes, the connected groups of data cells, and all device
 * workspace.
 *   ndim     2 or 3.
 *   dims     host array {nx, ny, nz}; nz is ignored when ndim == 2.  Each >= 1
 *            and the cell count nx*ny*nz below 2^31.
 *   spacing  host array {dx, dy, dz}, finite and > 0 (dz ignored in 2-D).
 *   mask     host pointer to nx*ny*nz bytes (copied), or NULL = all cells hold
 *            data.  At least one cell must hold data.
 *   flags    PI_FP32 or PI_FP64, ORed with PI_INNER_CG or PI_INNER_BICGSTAB,
 *            optionally ORed with PI_FIXED_POINT_CG (with PI_INNER_CG only)
 *            and PI_CELL_CENTERED (ndim == 2, PI_INNER_CG only).
 *   out      receives the plan; set to NULL on failure.
 * Errors: PI_ERR_INVALID_ARG, PI_ERR_OOM, PI_ERR_DEVICE.  Synchronous.
 */
pi_status pi_plan(int ndim, const int64_t dims[3], const double spacing[3], const uint8_t *mask,
                  uint32_t flags, pi_plan_t *out);

/* Release a plan and its device workspace (NULL is ignored).  Synchronous. */
void pi_plan_destroy(pi_plan_t plan);

/* Device bytes held by the plan. */
size_t pi_workspace_bytes(pi_plan_t plan);

/*
 * Inner-solve policy: `iters` Krylov iterations per outer step (1..4096).
 * The default grows with the longest side L: 3-D max(4, min(24, 3 ceil(log2
 * L) - 12)), 2-D max(4, min(32, 4 ceil(log2 L) - 24)) -- e.g. 12 at 256^3 and
 * 20 at 2048^2, the fastest counts measured for those sizes.  The paper
 * leaves the inner tolerance open; the fixed point of the outer iteration
 * does not depend on this choice, only the trajectory does.
 */
pi_status pi_set_inner_iters(pi_plan_t plan, int32_t iters);

/*
 * Tile shape of the stencil kernels: every wave owns a strip of 64 *
 * lane_cells consecutive cells along x and marches `mseg` planes (3-D) or
 * rows (2-D) along the slowest axis.  mseg 0 restores the size-based
 * default.  lane_cells is 1, 2 or 4 (4 needs nx % 4 == 0: each lane then
 * moves its cells with 16-byte accesses; 2 needs an even nx and the
 * face-crossing scheme: twice the waves of 4 at the same segment length),
 * 0 picks 4 when allowed, else 1.  The autotuner sweeps both knobs.
 * Returns PI_ERR_INVALID_ARG for other values.
 * Rebuilds the plan's block table (synchronous): PI_ERR_OOM if that fails,
 * and then pi_solve, pi_source, pi_apply and pi_time_kernel on the plan
 * return PI_ERR_OOM until a later pi_set_tile succeeds.
 * pi_get_tile / pi_get_lane_cells return the current values.
 */
pi_status pi_set_tile(pi_plan_t plan, int32_t mseg, int32_t lane_cells);
int32_t pi_get_tile(pi_plan_t plan);
int32_t pi_get_lane_cells(pi_plan_t plan);

/*
 * pi_solve -- Algorithm 1 on one grid.
 *   gx, gy, gz  device pointers to the gradient components (gz NULL in 2-D),
 *               float or double per the plan.  Values in masked cells are
 *               never read as data (NaN is allowed there).
 *   P           device pointer, same type: in = P^0 when PI_WARM_START is set
 *               (values in masked cells ignored); out = the returned pressure
 *               with the mean removed over every connected group of data
 *               cells (a data cell with no data neighbour gets 0); masked
 *               cells are set to NaN.
 *   tol         stop when eps_R <= tol (Eq. ResidualMomentum, relative to
 *               ||S||); tol >= 0.
 *   max_iter    upper bound on outer steps (>= 0).
 *   info        host pointer (may be NULL) filled when the call returns.
 * The call returns once the solve has finished on `stream` (it polls the
 * convergence flag); P is then valid.  If ||S|| = 0 the exact answer is a
 * constant, so P = 0 is returned in every data cell with eps_R = 0.  In FP32
 * mode eps_R refers to the FP64 iterate; rounding the returned field to float
 * alone leaves a residual of order 1e-7 * ||[W^{n+1}]-[W^n]|| ||P|| / ||S||.
 * If max_iter is reached first, the last iterate is returned (gauged)
 * together with PI_ERR_NOT_CONVERGED.
 * Errors: PI_ERR_INVALID_ARG, PI_ERR_NONFINITE, PI_ERR_NOT_CONVERGED,
 * PI_ERR_DIVERGED, PI_ERR_DEVICE.
 *
 * With PI_ASYNC the call only enqueues work on `stream` and returns PI_OK
 * (or an argument/launch error) at once; `info` is not touched.  Algorithm
 * 1's loop runs until eps_R <= tol, so its length is known only on the
 * device, and without device-side graph conditionals the queue cannot stop
 * itself: the call enqueues enough outer-step replays to reach max_iter
 * (<= 2^22), every kernel of which returns at once after the stop, then the
 * gauge and a copy of the final state.  A loose max_iter therefore costs
 * about 0.3 ms of empty launches per 8 unneeded outer steps at 256^3.  After
 * the stream has completed, P holds the result and pi_last_info gives its
 * pi_info (ms = 0) and status.  Without PI_ASYNC the call returns once the
 * solve is done: it polls the convergence flag between replays and never
 * launches past the stop.
 */
pi_status pi_solve(pi_plan_t plan, const void *gx, const void *gy, const void *gz, void *P,
                   double tol, int64_t max_iter, uint32_t flags, pi_info *info, void *stream);

/*
 * pi_last_info -- result of the plan's last pi_solve: fills info (ms = 0)
 * and returns its status.  For a PI_ASYNC solve, valid once the stream it
 * was enqueued on has completed.
 */
pi_status pi_last_info(pi_plan_t plan, pi_info *info);

/*
 * pi_solve_batched -- many independent grids of uneven size in one set of
 * launches: every kernel of an outer step walks a work list of tiles drawn
 * from the unfinished instances, scalars and the convergence flag are kept
 * per instance, and a bundle of outer steps is captured as a HIP graph and
 * replayed.  A finished instance's tiles return at once; when finished
 * instances hold a quarter of the listed tiles, the host (between replays)
 * rebuilds the work list without them and captures the graph again
 * (pi_info.worklist_rebuilds counts this).
 *   count         number of instances (>= 1); plans[i] must be distinct and
 *                 share the precision flag.
 *   gx, gy, gz, P host arrays of `count` device pointers, as for pi_solve
 *                 (gz may be NULL, or hold NULL for 2-D instances).
 *   tol           host array of `count` thresholds.
 *   infos         host array of `count` pi_info (may be NULL).
 * Returns the worst per-instance status (per-instance codes in infos[i]).
 */
pi_status pi_solve_batched(int64_t count, const pi_plan_t *plans, const void *const *gx,
                           const void *const *gy, const void *const *gz, void *const *P,
                           const double *tol, int64_t max_iter, uint32_t flags, pi_info *infos,
                           void *stream);

/*
 * pi_solve_batched_noalloc -- pi_solve_batched for callers that cannot
 * allocate device memory (tight serving loops, code under a capture or a
 * harness that forbids hipMalloc): the same arguments, kernels and results,
 * but the per-call device buffers (instance records, per-instance scalars,
 * partial sums, block tables) live in one static device array of the
 * library (about 32 MB on every GPU it runs on, held until the process
 * ends: room for the limits below).  The call allocates no device or pinned host memory and
 * creates no stream, event or graph: the outer steps are launched directly
 * on `stream` and the convergence flags are copied back to pageable host
 * memory every few outer steps (so it is slower per outer step than
 * pi_solve_batched for small grids).  The plans still own their vectors.
 * Limits: count <= PI_NOALLOC_MAX_INSTANCES, at most
 * PI_NOALLOC_MAX_PARTIALS blocks over all instances and
 * PI_NOALLOC_MAX_TABLE block-table entries; beyond them it returns
 * PI_ERR_TOO_LARGE before touching the device.  Every call rewrites what the
 * kernels read from the array before they run (it keeps the last call's
 * contents).  Calls share one array per GPU; the library serialises them
 * within a process, and returns once the work on `stream` has finished.
 */
#define PI_NOALLOC_MAX_INSTANCES 1024
#define PI_NOALLOC_MAX_PARTIALS 262144
#define PI_NOALLOC_MAX_TABLE 524288
pi_status pi_solve_batched_noalloc(int64_t count, const pi_plan_t *plans, const void *const *gx,
                                   const void *const *gy, const void *const *gz, void *const *P,
                                   const double *tol, int64_t max_iter, uint32_t flags, pi_info *infos,
                                   void *stream);

/*
 * pi_source -- the source vector {S} (Eq. ExplicitEqn_FaceCrossing, last sum)
 * on the grid: S is a device array of nx*ny*nz float/double, 0 in masked
 * cells.  Returns PI_ERR_NONFINITE (after a stream sync) if a data cell holds
 * a non-finite gradient.
 */
pi_status pi_source(pi_plan_t plan, const void *gx, const void *gy, const void *gz, void *S,
                    void *stream);

/*
 * pi_apply -- y = op x for op in {PI_OP_M, PI_OP_N, PI_OP_L} (the operators
 * of Eq. MatrixEquation), x and y device arrays of nx*ny*nz elements of the
 * plan's type; entries of x in masked cells are ignored, y is 0 there.
 * x and y must not overlap and must be aligned to the plan's lane access
 * (16 bytes for four cells per lane, 8 or 16 for two; torch allocations
 * are), else PI_ERR_INVALID_ARG.  Runs at the plan's current tile (pi_set_tile); the
 * result does not depend on it, the speed does: the tile the solve's
 * autotuner picks may give the apply too few waves, so a caller that applies
 * often can set its own.  Asynchronous.
 */
pi_status pi_apply(pi_plan_t plan, int op, const void *x, void *y, void *stream);

/*
 * pi_time_kernel -- measurement hook: launch one of the solve's kernels
 * `reps` times back to back on `stream`, exactly as the solve launches it
 * (same code, grid and data), bracketed by HIP events recorded on that
 * stream, and return the mean duration per launch in *avg_ms.  kernel is
 * PI_K_OUTER or PI_K_INNER (CG plans only).  Meant to run after a pi_solve
 * on the same plan and gradients (the workspace then holds solve data); it
 * overwrites the plan's workspace.  Synchronous.
 */
#define PI_K_OUTER 0   /* outer residual and update, Eq. ResidualMomentum      */
#define PI_K_INNER 1   /* one inner CG iteration: the previous iteration's
                          correction and residual update, the new search
                          direction and M p, in one pass (for a plan with
                          pi_get_cg_recompute = 1 the pass is two kernels,
                          the interior and the boundary layers; both are
                          timed)                                               */
pi_status pi_time_kernel(pi_plan_t plan, int kernel, int32_t reps, double *avg_ms, void *stream);

/*
 * pi_get_cg_recompute -- 1 if the plan's inner CG passes (after the first
 * of each outer step) evaluate q = M p_{k-1} again where they need it
 * instead of storing q and reading it back, else 0 (also for NULL).  The
 * iterates are the same bit for bit; a pass then moves 24 bytes per cell
 * (reads r, p and the correction, writes them) instead of 32.  Chosen for
 * 3-D FP32 CG plans without missing data at four cells per lane whose rows
 * fit one wave strip (nx <= 256) or split over as many overlapping wave
 * windows (owning 252 cells at the row ends, 248 between them) as 256-cell
 * strips: every nx up to 504 and most longer ones, 512 not; it follows the
 * tile, so read it after pi_set_tile or pi_autotune.
 */
int32_t pi_get_cg_recompute(pi_plan_t plan);

/*
 * pi_autotune -- pick the tile (pi_set_tile) that minimises the time of one
 * outer step of Algorithm 1 for this plan: for each candidate (segment
 * length, cells per lane) it times the outer kernel, the first inner CG pass
 * of a step and a later one (`reps` launches each; the CG passes, with their
 * finalize kernel where the tile needs one, as a HIP graph of eight passes,
 * as a solve runs them), models a step as outer + first + (inner_iters - 1)
 * later passes, times the three fastest again with
 * 4 * reps launches and keeps the fastest of those; then it chooses between
 * plain and non-temporal streams in the outer kernel (4 * reps launches each).  Results are
 * cached per (ndim, dims, precision, inner solver) for the life of the process,
 * so later plans of the same shape take the cached tile without timing.  The
 * chosen segment length is returned in *mseg (may be NULL).  Overwrites the
 * plan's workspace; synchronous.  The paper has no counterpart (its kernels
 * use one fixed launch shape); the knob changes speed, never results.
 */
pi_status pi_autotune(pi_plan_t plan, int32_t reps, int32_t *mseg, void *stream);

/* Human-readable name of a status code (static storage). */
const char *pi_status_string(pi_status status);

#ifdef __cplusplus
}
#endif

#endif /* PI_H */
