/*
 * fmg.h -- C interface of the MI355X (gfx950) solver for the 3D Poisson
 * equation L u = f, u = 0 on the boundary of the unit cube, by cell-centered
 * FAS full multigrid with optional segmental refinement.
 *
 * Method: Adams, Brown, Knepley, Samtaney, "Segmental Refinement: A Multigrid
 * Technique for Data Locality" (arXiv:1406.7808):
 *   - problem and cell-centered grid: Sec. 2, Eqs. (1)-(2);
 *   - FAS V-cycle: Sec. 3.1, Eqs. (3)-(4), Fig. 1;
 *   - full multigrid F(alpha, nu1, nu2): Sec. 3.2, Fig. 2;
 *   - segmental refinement: Sec. 4, Eq. (5), Figs. 5-6.
 * Discretization and transfers: 7-point Laplacian, red-black Gauss-Seidel
 * (red = (i+j+k) even, red first), mean-of-8 restriction, piecewise-constant
 * V-cycle prolongation, trilinear FMG interpolation, exact coarsest solve.
 *
 * Conventions for every entry point:
 *   - Grids are N^3 contiguous double arrays in DEVICE memory, element
 *     [(k*N + j)*N + i] is cell (i,j,k) with center ((i+1/2)h, (j+1/2)h,
 *     (k+1/2)h), h = 1/N (x fastest; a torch tensor of shape (N,N,N) indexed
 *     [z,y,x]).
 *   - `stream` is a hipStream_t passed as void* (NULL = default stream); work
 *     is enqueued asynchronously on it and no call synchronizes the device
 *     except fmg_plan_create/destroy and fmg_solve.
 *   - Return value: FMG_OK (0) or a negative fmg_status; the message of the
 *     last failure on the calling thread is returned by fmg_last_error().
 *     Parameter errors are detected on the host before anything is enqueued.
 *     Nothing aborts the process.
 */
#ifndef FMG_H
#define FMG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FMG_OK = 0,
  FMG_EINVAL = -1, /* invalid argument (shape, schedule, pointer) */
  FMG_ENOMEM = -2, /* device allocation failed */
  FMG_EHIP = -3,   /* a HIP runtime call failed */
  FMG_ENOTSUP = -4 /* valid but unsupported combination */
} fmg_status;

typedef enum {
  FMG_FP64 = 0,        /* every operation in FP64 */
  FMG_FP32_REFINED = 1 /* FP32 multigrid corrected by FP64 residuals */
} fmg_precision;

/*
 * Solver parameters.
 *   levels            total number of grids M+1 (Sec. 2): level 0 is the
 *                     coarsest, edge n0 = N >> (levels-1), with
 *                     n0 << (levels-1) == N and 1 <= n0 <= 8.
 *   sr_levels         K: the K finest levels are solved by segmental
 *                     refinement (Sec. 4); 0 = plain global FMG.
 *                     0 <= K <= levels-1.  The transition level is
 *                     T = levels-1-K.
 *   segments_per_dim  S >= 1 segments per dimension (S^3 segments); needs
 *                     N % (S << K) == 0 so that every segment owns at least
 *                     one cell of the transition level.
 *   buffer_schedule   HOST pointer to K buffer widths J, FINEST LEVEL FIRST
 *                     (J for level levels-1, then levels-2, ...), each even
 *                     and >= 0 (Eq. 5), and each at least half the width of
 *                     the next finer level (the coarse support of a compute
 *                     region must lie inside the coarser compute region).
 *                     May be NULL when K == 0.  Copied at plan creation.
 *   nu_pre, nu_post, alpha
 *                     red-black sweeps before and after the coarse-grid
 *                     correction and after each FMG interpolation (the
 *                     F(alpha, nu1, nu2) cycle of Sec. 3.2); each 0..8.
 *   precision         fmg_precision.
 *   refine_iters      FP64 residual corrections for FMG_FP32_REFINED (0..8).
 */
typedef struct {
  int32_t levels;
  int32_t sr_levels;
  int32_t segments_per_dim;
  const int32_t *buffer_schedule;
  int32_t nu_pre, nu_post, alpha;
  int32_t precision;
  int32_t refine_iters;
} fmg_params;

typedef struct fmg_plan fmg_plan;

/* Host-only validation of (N, *p); no device call.  FMG_OK or FMG_EINVAL.
 * The rules: the level hierarchy of Sec. 2 (N = n0 * 2^(levels-1)), the
 * segment and buffer-width conditions of Sec. 4 (Eq. 5: even widths; each at
 * least half the next finer one, so that a compute region's coarse support
 * lies in the coarser compute region), sweep counts of the F(alpha, nu1, nu2)
 * cycle of Sec. 3.2. */
int32_t fmg_check_params(int32_t N, const fmg_params *p);

/* Validate, select `device`, allocate all device workspace and precompute the
 * coarsest-level inverse (in FP64 on the host; the exact coarsest solve of
 * Fig. 1 and Fig. 2).  The workspace holds the global levels of Sec. 3 and
 * the segment-private boxes (compute region plus frozen ghosts) of Sec. 4.
 * On success *out owns the workspace until fmg_plan_destroy.  FMG_EINVAL,
 * FMG_ENOMEM or FMG_EHIP on failure (then *out is NULL). */
int32_t fmg_plan_create(int32_t N, const fmg_params *p, int32_t device, fmg_plan **out);

/* Enqueue one solve on `stream`: u <- FMG(f) (Fig. 2 for sr_levels == 0,
 * Fig. 5 otherwise).  f, u: device pointers to N^3 doubles; u is fully
 * overwritten (its prior content is ignored); f is read only and must stay
 * valid until the stream passes the solve.  f and u must not overlap.  A plan
 * serves one stream at a time and is not thread-safe. */
int32_t fmg_plan_execute(fmg_plan *plan, const double *f, double *u, void *stream);

/*
 * Performance knobs of a plan.  Every valid setting computes the same solve
 * (results agree to rounding: the smoothers differ only in forming
 * 1/(6 + b_c) products and the order of a few sums); the batched interface
 * and the autotuner pick them per problem size.
 *   max_stages     half-sweeps per pass of the streaming smoother on levels
 *                  smoothed over two copies: 2 or 4 (default 4);
 *   seg_inplace    1: segment levels whose compute region plus an 8-cell halo
 *                  fits 2048 columns are smoothed in place, one workgroup per
 *                  segment, 4 half-sweeps per pass (default 1);
 *   box            1: segment levels whose whole storage box fits the LDS of
 *                  one workgroup use the box-resident smoother (default 1);
 *   target_blocks  workgroups a streaming pass aims for, 64..65536, or 0
 *                  (default): on levels above 64^3 the z chunks of each
 *                  pass over two copies are chosen for the fewest rounds of
 *                  resident workgroups times chunk depth, elsewhere 1024;
 *   tile_x         width in columns of the xy tiles of the streaming passes
 *                  over two copies: even, 8..256 (clamped per pass to what
 *                  its halo and workgroup admit; the height follows from the
 *                  workgroup's columns), or 0 (default): the shape that loads
 *                  the fewest columns.
 * fmg_plan_set_tuning re-plans the schedule on the host (no device call);
 * FMG_EINVAL for out-of-range values.
 */
typedef struct {
  int32_t max_stages;
  int32_t seg_inplace;
  int32_t box;
  int32_t target_blocks;
  int32_t tile_x;
} fmg_tuning;

int32_t fmg_plan_get_tuning(const fmg_plan *plan, fmg_tuning *out);
int32_t fmg_plan_set_tuning(fmg_plan *plan, const fmg_tuning *tuning);

/* Level checkpoints (the per-level state of the differentiable solve, and a
 * validation hook): while set, every fmg_plan_execute also writes the
 * solution of each level l right after its FMG stage (Fig. 2: after the
 * stage's V-cycle; Fig. 5 for segment levels, whose genuine cells are
 * written) into out[l], a DEVICE array of n_l^3 doubles with
 * n_l = N >> (levels - 1 - l) in the layout above.  out is a HOST array of
 * `levels` such pointers (NULL entries are skipped), copied at the call; the
 * arrays must stay valid while set.  out == NULL clears them.  FP64 plans
 * only (FMG_ENOTSUP otherwise). */
int32_t fmg_plan_checkpoints(fmg_plan *plan, double *const *out);

/* The comparison solver of Sec. 7 (Fig. 10): V(nu_pre, nu_post) cycles
 * (Fig. 1) on the plan's hierarchy, starting from the guess in u, until
 * max_c |f - L_h u|_c <= rtol * max_c |f_c| or maxit cycles; u (device, N^3)
 * is updated in place.  *iters and *relres (host, may be NULL) receive the
 * cycle count and the final max|f - L u| / max|f|.  Global FP64 plans only
 * (sr_levels == 0): FMG_ENOTSUP otherwise.  Synchronizes `stream` once per
 * cycle (the stopping test); rtol == 0 runs exactly maxit cycles and forms
 * the residual once, after the last (nothing waits between cycles); rtol == 0
 * with relres == NULL forms no residual and never synchronizes, so the call
 * only enqueues work and may be captured into a HIP graph.  The norm
 * partials live in the plan's workspace: the call allocates nothing.
 * FMG_EINVAL for null or overlapping f/u, rtol < 0, maxit < 0, or a residual
 * that is not finite (NaN or Inf in f or u). */
int32_t fmg_plan_vcycles(fmg_plan *plan, const double *f, double *u, double rtol, int32_t maxit,
                         int32_t *iters, double *relres, void *stream);

/* Free the workspace (synchronizes the plan's device).  NULL is accepted. */
int32_t fmg_plan_destroy(fmg_plan *plan);

/* create + execute + stream synchronize + destroy: one solve of Fig. 2
 * (sr_levels == 0) or Fig. 5, with the arguments, layout and errors of
 * fmg_plan_create and fmg_plan_execute; allocates and frees the workspace. */
int32_t fmg_solve(const double *f, int32_t N, const fmg_params *p, double *u, void *stream);

/* Device bytes held by the plan. */
int64_t fmg_plan_workspace_bytes(const fmg_plan *plan);

/*
 * Kernel timing.  While enabled, every launch enqueued by fmg_plan_execute
 * is bracketed by two HIP events on the solve's stream; fmg_plan_profile_read
 * waits for the last one, aggregates per kernel name and level ("name@level",
 * level 0 = coarsest; no suffix for whole-grid steps) and clears the records.
 * `bytes` sums the algorithmic bytes of the launches: the cells each launch
 * must read and write at least once (one read of every input cell it uses, one
 * write of every output cell), independent of caching.
 */
typedef struct {
  char name[64];
  int64_t launches;
  double total_ms;
  double bytes;
} fmg_kernel_stat;

/* Enable (1) or disable (0) timing; pending records are discarded. */
int32_t fmg_plan_profile(fmg_plan *plan, int32_t enable);

/* Copy up to `cap` per-kernel aggregates to out and their number to *count
 * (synchronizes with the last timed launch). */
int32_t fmg_plan_profile_read(fmg_plan *plan, fmg_kernel_stat *out, int32_t cap, int32_t *count);

/*
 * Schedule model (host only, no device call): walks the launches of one
 * fmg_plan_execute for (N, *p) on a virtual workspace, checking every
 * launch's pointers and grid, and returns the launch count, the sum of their
 * algorithmic bytes (as in fmg_kernel_stat) and the workspace a plan would
 * allocate.
 */
typedef struct {
  int64_t launches;
  double bytes;
  int64_t workspace_bytes;
} fmg_schedule_stat;

int32_t fmg_schedule_model(int32_t N, const fmg_params *p, fmg_schedule_stat *out);

/*
 * Norms (the quantities Sec. 7 reports in Figs. 8 and 10), by wavefront
 * reduction on the device.  f, u, v: device arrays of N^3 doubles (layout as
 * above); out: HOST array of 2 doubles.  Both calls allocate a small temporary
 * device buffer and synchronize `stream` before returning.
 *   fmg_residual_norms: r = f - L_h u (7-point operator of Eq. 2);
 *   fmg_diff_norms:     r = u - v;
 *   out[0] = max_c |r_c|,  out[1] = sqrt(h^3 sum_c r_c^2)  (h = 1/N: the L2
 *   norm of the cellwise-constant function on the unit cube).
 * FMG_EINVAL for null pointers, N < 1 or f == u; FMG_ENOMEM / FMG_EHIP.
 */
int32_t fmg_residual_norms(const double *f, const double *u, int32_t N, double *out,
                           void *stream);
int32_t fmg_diff_norms(const double *u, const double *v, int32_t N, double *out, void *stream);

/* fmg_residual_norms for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * kernels and results, but the partial sums live in a static device array of
 * 1024 pairs of doubles (16 KiB per GPU, held until the process ends), out is
 * a DEVICE array of 2 doubles, and the call only enqueues two kernels on
 * `stream`: no allocation, no copy, no synchronization.  Any N in 1..4096 fits
 * (the reduction strides over the grid); larger N is FMG_EINVAL.  Calls that
 * overlap on one GPU (other streams or threads) share the array and race;
 * serialize them.  FMG_EINVAL for null pointers or f == u; FMG_EHIP. */
int32_t fmg_residual_norms_noalloc(const double *f, const double *u, int32_t N, double *out,
                                   void *stream);


/*
 * Batches of independent solves (sizes, parameters and tunings may differ).
 * The problems are spread over `streams` internal streams (1..16; longest
 * first, each to the least loaded stream) so that small solves run side by
 * side; problems sharing a stream and equal (N, params, tuning) share one
 * plan's workspace.
 *   fmg_batch_create: count problems; N, params (and tuning, or NULL for the
 *     defaults) are HOST arrays of `count` entries, copied at the call.
 *   fmg_batch_execute: u[i] <- FMG(f[i]) for every problem; f and u are HOST
 *     arrays of `count` device pointers (N[i]^3 doubles each, layout above;
 *     no u[i] may overlap another problem's f or u).  The call forks `stream`
 *     to the internal streams and joins them back, so later work on `stream`
 *     sees every solution.
 *   fmg_batch_capture: records the same work for these pointers into a HIP
 *     graph owned by the batch (replacing an earlier one); `stream` must not
 *     be the legacy default stream.  fmg_batch_replay launches that graph:
 *     the whole batch in one graph launch.
 * FMG_EINVAL on a parameter error (with the problem's index in the message).
 */
typedef struct fmg_batch fmg_batch;

int32_t fmg_batch_create(int32_t count, const int32_t *N, const fmg_params *params,
                         const fmg_tuning *tuning, int32_t streams, int32_t device,
                         fmg_batch **out);
int32_t fmg_batch_execute(fmg_batch *batch, const double *const *f, double *const *u,
                          void *stream);
int32_t fmg_batch_capture(fmg_batch *batch, const double *const *f, double *const *u,
                          void *stream);
int32_t fmg_batch_replay(fmg_batch *batch, void *stream);
int64_t fmg_batch_workspace_bytes(const fmg_batch *batch);
int32_t fmg_batch_destroy(fmg_batch *batch);

/* Message of the last non-OK status returned on this thread ("" if none). */
const char *fmg_last_error(void);

/*
 * Single operators on one whole level of edge n (device arrays of n^3
 * doubles, layout as above), enqueued on `stream`.  They run the same
 * kernels as the solver and exist to test them one by one.
 *   fmg_op_apply:    out = L_h u                      (Eq. 2, 7-point)
 *   fmg_op_smooth:   nu red-black Gauss-Seidel sweeps on u for L_h u = rhs
 *                    (allocates a temporary copy of u and synchronizes
 *                    `stream` before returning)
 *   fmg_op_restrict: coarse ((n/2)^3) = mean of the 8 children of fine (n^3)
 *   fmg_op_interp:   fine ((2n)^3) = trilinear FMG interpolation of coarse
 *                    (n^3), odd reflection at the walls (Sec. 3.2)
 */
int32_t fmg_op_apply(const double *u, int32_t n, double *out, void *stream);
int32_t fmg_op_smooth(double *u, const double *rhs, int32_t n, int32_t nu, void *stream);
int32_t fmg_op_restrict(const double *fine, int32_t n, double *coarse, void *stream);
int32_t fmg_op_interp(const double *coarse, int32_t n, double *fine, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* FMG_H */
