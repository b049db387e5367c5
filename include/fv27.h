/*
 * fv27.h -- C interface of the MI355X (gfx950) solver for the paper's own
 * model problem: the Laplacian on a box of cubic cells (the paper's
 * [0,2] x [0,1]^2), zero Dirichlet boundary, by cell-centered FAS full
 * multigrid with optional segmental refinement.
 *
 * Method: Adams, Brown, Knepley, Samtaney, "Segmental Refinement: A Multigrid
 * Technique for Data Locality" (arXiv:1406.7808):
 *   - model problem and solver: Sec. 5.1 (27-point finite volume stencil of
 *     second order, piecewise constant restriction, linear prolongation for
 *     both the FMG and the V-cycle prolongation, second degree Chebyshev
 *     pre- and post-smoothers, a first degree Chebyshev smoother after each
 *     FMG prolongation: the F(1,2,2) cycle);
 *   - FAS V-cycle and FMG: Sec. 3, Figs. 1-2; segmental refinement: Sec. 4,
 *     Eq. (5), Figs. 5-6; buffer schedules of the experiments: Sec. 5.2.
 * Discretization (where the paper gives no formula):
 *   - operator: each cell's balance of its six face fluxes; a face flux is
 *     the face average of the normal difference quotient over the 3 x 3 cell
 *     columns touching the face, with weights 1/24, 11/12, 1/24 per
 *     transverse dimension (27-point stencil, h^-2 sum_d D2_d W_e W_f);
 *     ghost cells beyond a wall hold the odd reflection of the interior;
 *   - Chebyshev smoother of degree k: k steps u <- u - (rhs - L u) / (d l_j),
 *     d = (121/24) h^-2, l_j the roots of the degree-k Chebyshev polynomial
 *     of [48/121, 200/121] (the stencil's symbol on the modes a grid twice
 *     as coarse cannot represent), l_j = 124/121 + (76/121) cos((2j-1) pi/(2k));
 *   - restriction: mean of 8 children; prolongation: trilinear, odd
 *     reflection at walls; coarsest level: exact (dense inverse).
 *
 * Conventions (as in fmg.h): grids are DEVICE arrays of n0*n1*n2 doubles,
 * element [(k*n1 + j)*n0 + i] is cell (i,j,k) with center ((i+1/2)h,
 * (j+1/2)h, (k+1/2)h); `stream` is a hipStream_t passed as void*; calls
 * return 0 or a negative status of fmg.h's fmg_status (FMG_EINVAL, FMG_ENOMEM,
 * FMG_EHIP); fv27_last_error() gives the message of the last failure on the
 * calling thread.  Parameter errors are detected on the host before any
 * launch; nothing aborts.
 */
#ifndef FV27_H
#define FV27_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/*
 * Solver parameters.
 *   n                finest extents (cells per dimension, x first); the
 *                    paper's grid is 4g x 2g x 2g for a 4 x 2 x 2 process grid
 *                    of g^3 cells each.
 *   h                finest cell size (> 0); the domain is [0, n[d] h].
 *   levels           total levels; every n[d] divisible by 2^(levels-1); the
 *                    coarsest level (extents n[d] >> (levels-1)) has at most
 *                    512 cells and is solved exactly.
 *   sr_levels        K in [0, levels-1]: the K finest levels are solved by
 *                    segmental refinement (Sec. 4); 0 = plain global FMG.
 *   segments         segments per dimension, each >= 1, with n[d] divisible
 *                    by segments[d] << K and n[d] / segments[d] equal for all
 *                    d (cubic segments, the paper's process subdomains).
 *   buffer_schedule  HOST pointer to K buffer widths, FINEST LEVEL FIRST, each
 *                    even and >= 0 and each at least half the next finer one
 *                    (Eq. 5 gives J_k = 2 floor((A + B (K - k)) / 2)); may be
 *                    NULL when K == 0.  Copied at plan creation.
 *   cheb_pre, cheb_post, cheb_fmg
 *                    Chebyshev degrees of the pre- and post-smoother and of
 *                    the smoother after each FMG prolongation, each 0..8
 *                    (the paper's F(1,2,2): 2, 2, 1).
 */
typedef struct {
  int32_t n[3];
  double h;
  int32_t levels;
  int32_t sr_levels;
  int32_t segments[3];
  const int32_t *buffer_schedule;
  int32_t cheb_pre, cheb_post, cheb_fmg;
} fv27_params;

typedef struct fv27_plan fv27_plan;

/* Host-only validation of *p (the hierarchy of Sec. 2 on a box, the segment
 * and buffer conditions of Sec. 4 and Eq. 5); 0 or FMG_EINVAL. */
int32_t fv27_check_params(const fv27_params *p);

/* Validate, select `device`, allocate the workspace (global levels; per SR
 * level one storage box per segment covering its compute region plus a ghost
 * layer, Sec. 4) and form the coarsest level's inverse on the host in FP64.
 * *out owns the workspace until fv27_plan_destroy.  FMG_EINVAL, FMG_ENOMEM or
 * FMG_EHIP (then *out is NULL). */
int32_t fv27_plan_create(const fv27_params *p, int32_t device, fv27_plan **out);

/* Enqueue one solve on `stream`: u <- FMG(f) (Fig. 2 when sr_levels == 0,
 * Figs. 5-6 otherwise).  f, u: device arrays of n0*n1*n2 doubles, must not
 * overlap; u is fully overwritten; f must stay valid until the stream passes
 * the solve.  Allocates nothing and does not synchronize.  A plan serves one
 * stream at a time. */
int32_t fv27_plan_execute(fv27_plan *plan, const double *f, double *u, void *stream);

/* Free the workspace (synchronizes the plan's device); NULL is accepted. */
int32_t fv27_plan_destroy(fv27_plan *plan);

/* Device bytes held by the plan. */
int64_t fv27_plan_workspace_bytes(const fv27_plan *plan);

/* Launches of one execute and the sum of their algorithmic bytes (each input
 * cell a launch needs read once, each output cell written once). */
int32_t fv27_plan_model(const fv27_plan *plan, int64_t *launches, double *bytes);

/* Single operators on a whole box of extents n, cell size h (device arrays),
 * enqueued on `stream`; they run the solver's kernels, for tests:
 *   fv27_op_apply: out = L_h u (the 27-point operator);
 *   fv27_op_cheb:  degree-k Chebyshev smoothing of L_h u = rhs, in place
 *                  (allocates a temporary copy, synchronizes `stream`);
 *   fv27_op_prolong: fine (2n) = trilinear prolongation of coarse (n). */
int32_t fv27_op_apply(const double *u, const int32_t *n, double h, double *out, void *stream);
int32_t fv27_op_cheb(double *u, const double *rhs, const int32_t *n, double h, int32_t degree,
                     void *stream);
int32_t fv27_op_prolong(const double *coarse, const int32_t *n, double *fine, void *stream);

/* Message of the last failure of an fv27_* call on this thread ("" if none). */
const char *fv27_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FV27_H */
