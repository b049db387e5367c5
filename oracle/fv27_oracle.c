/*
 * fv27_oracle.c -- plain FP64 CPU oracle for the paper's own model problem
 * (Adams, Brown, Knepley, Samtaney, "Segmental Refinement: A Multigrid
 * Technique for Data Locality", arXiv:1406.7808, Sec. 5.1): cell-centered
 * FAS full multigrid, with and without segmental refinement, for the
 * Laplacian on a box of cubic cells, zero Dirichlet boundary, 27-point
 * finite volume operator, Chebyshev polynomial smoothers and linear
 * prolongation.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the HIP library in paper_1406_7808_amd/csrc.
 *
 * Every grid access goes through a bounds-checked accessor and every region
 * is the paper's set definition written out; OpenMP only splits loops whose
 * iterations are independent, so results do not depend on the thread count.
 *
 * Model problem (Sec. 5.1): L u = f with L the Laplacian on the box
 * [0, n0 h] x [0, n1 h] x [0, n2 h] (the paper's [0,2] x [0,1]^2), u = 0 on
 * the boundary.  The solver there uses piecewise constant restriction, linear
 * prolongation for both the FMG and the V-cycle prolongation, second degree
 * Chebyshev pre- and post-smoothers and a first degree Chebyshev smoother
 * after each FMG prolongation (the F(1,2,2) cycle), and a 27-point finite
 * volume stencil of second order.  Readings where the paper says no more:
 *   - operator: the finite volume balance of the six face fluxes of a cell;
 *     a face flux is the face average of the normal derivative, taken as
 *     the centered difference across the face in each of the 3 x 3 cell
 *     columns that touch the face, averaged with the weights of the
 *     quadratic interpolant integrated over the face: 1/24, 11/12, 1/24 per
 *     transverse dimension (the cell's own column gets 11/12).  This gives a
 *     27-point stencil; on every cell row it equals
 *       h^-2 sum_d D2_d W_e W_f,  D2 = (1,-2,1), W = (1/24, 11/12, 1/24);
 *   - boundary: ghost cells beyond a wall hold the odd reflection of the
 *     interior value (linear interpolation to zero on the face, Sec. 3.3),
 *     per dimension, so edge and corner ghosts carry the product of signs;
 *   - smoother: Chebyshev iteration for A = -L with the scalar preconditioner
 *     1/d, d = (121/24) h^-2 the magnitude of the stencil's centre weight.
 *     The sine modes at cell centres are eigenvectors of L on the box (both
 *     1D factors are), so the spectrum of A/d is the stencil's symbol
 *     sampled at the grid frequencies, inside (0, 200/121].  The smoother
 *     targets the modes that a grid twice as coarse cannot represent (some
 *     frequency >= pi/2), where the symbol lies in [48/121, 200/121].  A
 *     degree-k smoother is the Chebyshev polynomial of that interval,
 *     normalized to 1 at zero, applied as k Jacobi-type steps
 *       u <- u - (1 / (d lambda_j)) (rhs - L u)   on the compute region,
 *     one per root lambda_j = (a+b)/2 + (b-a)/2 cos((2j-1) pi / (2k)),
 *     j = 1..k, [a, b] = [48/121, 200/121];
 *   - restriction of solution and residual: mean of the 8 children;
 *   - prolongation (FMG and V-cycle): trilinear, 1D weights 3/4 and 1/4
 *     toward the nearer coarse neighbour, coarse values beyond a wall by odd
 *     reflection;
 *   - FMG right-hand sides f_{l-1} = R f_l; coarsest level: exact dense
 *     solve (LU with partial pivoting);
 *   - segmental refinement as in Figs. 5 and 6 with segments as a
 *     s0 x s1 x s2 array of equal boxes of cubic genuine regions (the
 *     paper's 4 x 2 x 2 process grid), the level-(k-1) regions of Fig. 6 read
 *     as F_{k-1} = C_k / 2, and the transition level written once per cell,
 *     restricted from the segment whose genuine region covers it.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* grids                                                                     */
/* ------------------------------------------------------------------------ */

typedef struct {
  int n[3];   /* level extents: the domain is cells [0,n0) x [0,n1) x [0,n2) */
  double h;   /* cell size of this level */
  int lo[3];  /* level index of storage element (0,0,0) */
  int ext[3]; /* storage extent per dimension */
  double *v;  /* values, x fastest */
} grid;

typedef struct {
  int n[3];
  double h;
} level;

static void die(const char *msg) {
  fprintf(stderr, "fv27_oracle: %s\n", msg);
  abort();
}

static grid grid_new(const level *lv, const int lo[3], const int hi[3]) {
  grid g;
  for (int d = 0; d < 3; ++d) {
    g.n[d] = lv->n[d];
    g.lo[d] = lo[d];
    g.ext[d] = hi[d] - lo[d];
    if (g.ext[d] <= 0) die("empty grid");
  }
  g.h = lv->h;
  size_t cnt = (size_t)g.ext[0] * g.ext[1] * g.ext[2];
  g.v = (double *)calloc(cnt, sizeof(double));
  if (!g.v) die("out of memory");
  return g;
}

static grid grid_level(const level *lv) {
  int lo[3] = {0, 0, 0};
  return grid_new(lv, lo, lv->n);
}

static void grid_free(grid *g) {
  free(g->v);
  g->v = NULL;
}

static size_t grid_count(const grid *g) { return (size_t)g->ext[0] * g->ext[1] * g->ext[2]; }

static void copy_grid(grid *dst, const grid *src) {
  if (grid_count(dst) != grid_count(src)) die("copy between grids of different size");
  memcpy(dst->v, src->v, sizeof(double) * grid_count(src));
}

static inline size_t at(const grid *g, int i, int j, int k) {
  int a = i - g->lo[0], b = j - g->lo[1], c = k - g->lo[2];
  if (a < 0 || b < 0 || c < 0 || a >= g->ext[0] || b >= g->ext[1] || c >= g->ext[2]) {
    fprintf(stderr, "fv27_oracle: access (%d,%d,%d) outside box lo=(%d,%d,%d) ext=(%d,%d,%d)\n",
            i, j, k, g->lo[0], g->lo[1], g->lo[2], g->ext[0], g->ext[1], g->ext[2]);
    abort();
  }
  return ((size_t)c * g->ext[1] + b) * g->ext[0] + a;
}

static inline double get(const grid *g, int i, int j, int k) { return g->v[at(g, i, j, k)]; }
static inline void put(grid *g, int i, int j, int k, double x) { g->v[at(g, i, j, k)] = x; }

static inline int in_domain(const int n[3], int i, int j, int k) {
  return i >= 0 && j >= 0 && k >= 0 && i < n[0] && j < n[1] && k < n[2];
}

/* a region [a, b) of cells in level indices */
typedef struct {
  int a[3], b[3];
} region;

static region whole(const int n[3]) {
  region r = {{0, 0, 0}, {n[0], n[1], n[2]}};
  return r;
}

static inline int in_region(const region *r, int i, int j, int k) {
  return i >= r->a[0] && i < r->b[0] && j >= r->a[1] && j < r->b[1] && k >= r->a[2] &&
         k < r->b[2];
}

static int floordiv2(int i) { return (i >= 0) ? i / 2 : -((-i + 1) / 2); }

/* odd reflection of one index across the walls of [0, n): returns the sign */
static int reflect(int n, int *i) {
  if (*i < 0) {
    *i = -1 - *i;
    return -1;
  }
  if (*i >= n) {
    *i = 2 * n - 1 - *i;
    return -1;
  }
  return 1;
}

/* value of cell (i,j,k) of g, a ghost beyond a wall being the odd reflection
 * of the interior cell (per dimension); cells inside the domain are read from
 * storage (for a segment: its compute region or its frozen ghost layer) */
static double value(const grid *g, int i, int j, int k) {
  int idx[3] = {i, j, k};
  int sign = 1;
  for (int d = 0; d < 3; ++d) sign *= reflect(g->n[d], &idx[d]);
  return (double)sign * get(g, idx[0], idx[1], idx[2]);
}

/* ------------------------------------------------------------------------ */
/* the 27-point finite volume operator (Sec. 5.1)                            */
/* ------------------------------------------------------------------------ */

/* face-average weights of the 3 cell columns across a face, per transverse
 * dimension (offset -1, 0, +1): the quadratic interpolant through the three
 * column values, integrated over the face width */
static const double FACE_W[3] = {1.0 / 24.0, 11.0 / 12.0, 1.0 / 24.0};

/* flux through the face of cell (i,j,k) on side s = +-1 of dimension d:
 * face average of (u_outside - u_inside) / h over the 3 x 3 columns */
static double face_flux(const grid *u, int i, int j, int k, int d, int s) {
  int e = (d + 1) % 3, f = (d + 2) % 3;
  double sum = 0.0;
  for (int b = -1; b <= 1; ++b)
    for (int a = -1; a <= 1; ++a) {
      int in[3] = {i, j, k};
      in[e] += a;
      in[f] += b;
      int out[3] = {in[0], in[1], in[2]};
      out[d] += s;
      double diff = value(u, out[0], out[1], out[2]) - value(u, in[0], in[1], in[2]);
      sum += FACE_W[a + 1] * FACE_W[b + 1] * diff;
    }
  return sum / u->h;
}

/* (L_h u)_c = (sum of the 6 outward face fluxes) / h: the cell balance of
 * the finite volume method divided by the cell volume h^3 (face area h^2) */
static double apply_L(const grid *u, int i, int j, int k) {
  double s = 0.0;
  for (int d = 0; d < 3; ++d) {
    s += face_flux(u, i, j, k, d, +1);
    s += face_flux(u, i, j, k, d, -1);
  }
  return s / u->h;
}

/* res = rhs - L u over region r */
static void residual(grid *res, const grid *u, const grid *rhs, const region *r) {
#pragma omp parallel for schedule(static)
  for (int k = r->a[2]; k < r->b[2]; ++k)
    for (int j = r->a[1]; j < r->b[1]; ++j)
      for (int i = r->a[0]; i < r->b[0]; ++i)
        put(res, i, j, k, get(rhs, i, j, k) - apply_L(u, i, j, k));
}

/* ------------------------------------------------------------------------ */
/* Chebyshev smoother                                                        */
/* ------------------------------------------------------------------------ */

static const double CHEB_A = 48.0 / 121.0;  /* symbol of A/d on the modes the coarse grid misses */
static const double CHEB_B = 200.0 / 121.0; /* the symbol's maximum */

/* root j (1..k) of the degree-k Chebyshev polynomial of [a, b] */
static double cheb_root(int j, int k) {
  const double pi = 3.14159265358979323846;
  return 0.5 * (CHEB_A + CHEB_B) + 0.5 * (CHEB_B - CHEB_A) * cos((2.0 * j - 1.0) * pi / (2.0 * k));
}

/* degree-k Chebyshev smoothing of L u = rhs on region r: k Jacobi-type
 * steps, each from the residual of the previous iterate (cells outside r,
 * frozen ghosts included, are read and never written) */
static void cheb_smooth(grid *u, const grid *rhs, const region *r, int k) {
  if (k <= 0) return;
  int lo[3], hi[3];
  for (int d = 0; d < 3; ++d) {
    lo[d] = r->a[d];
    hi[d] = r->b[d];
  }
  level lv = {{u->n[0], u->n[1], u->n[2]}, u->h};
  grid res = grid_new(&lv, lo, hi);
  const double d = (121.0 / 24.0) / (u->h * u->h);
  for (int j = 1; j <= k; ++j) {
    residual(&res, u, rhs, r);
    const double c = 1.0 / (d * cheb_root(j, k));
#pragma omp parallel for schedule(static)
    for (int kk = r->a[2]; kk < r->b[2]; ++kk)
      for (int jj = r->a[1]; jj < r->b[1]; ++jj)
        for (int ii = r->a[0]; ii < r->b[0]; ++ii)
          put(u, ii, jj, kk, get(u, ii, jj, kk) - c * get(&res, ii, jj, kk));
  }
  grid_free(&res);
}

/* ------------------------------------------------------------------------ */
/* transfers                                                                 */
/* ------------------------------------------------------------------------ */

/* coarse cell = mean of its 8 children */
static double restrict_cell(const grid *fine, int I, int J, int K) {
  double s = 0.0;
  for (int c = 0; c < 2; ++c)
    for (int b = 0; b < 2; ++b)
      for (int a = 0; a < 2; ++a) s += get(fine, 2 * I + a, 2 * J + b, 2 * K + c);
  return s / 8.0;
}

/* trilinear prolongation: value at fine cell (i,j,k) from coarse grid c */
static double prolong_cell(const grid *c, int i, int j, int k) {
  int fi[3] = {i, j, k};
  int p[3], q[3];
  for (int d = 0; d < 3; ++d) {
    p[d] = floordiv2(fi[d]);
    q[d] = (fi[d] - 2 * p[d] == 0) ? p[d] - 1 : p[d] + 1; /* the other neighbour */
  }
  double s = 0.0;
  for (int cz = 0; cz < 2; ++cz)
    for (int cy = 0; cy < 2; ++cy)
      for (int cx = 0; cx < 2; ++cx) {
        double w = (cx ? 0.25 : 0.75) * (cy ? 0.25 : 0.75) * (cz ? 0.25 : 0.75);
        s += w * value(c, cx ? q[0] : p[0], cy ? q[1] : p[1], cz ? q[2] : p[2]);
      }
  return s;
}

/* ------------------------------------------------------------------------ */
/* coarsest level: exact dense solve                                         */
/* ------------------------------------------------------------------------ */

static void coarse_solve(grid *u, const grid *rhs) {
  const int *n = u->n;
  int m = n[0] * n[1] * n[2];
  double *A = (double *)calloc((size_t)m * m, sizeof(double));
  double *x = (double *)calloc((size_t)m, sizeof(double));
  if (!A || !x) die("out of memory");
  level lv = {{n[0], n[1], n[2]}, u->h};
  grid e = grid_level(&lv);
  for (int col = 0; col < m; ++col) {
    memset(e.v, 0, sizeof(double) * m);
    e.v[col] = 1.0;
    for (int k = 0; k < n[2]; ++k)
      for (int j = 0; j < n[1]; ++j)
        for (int i = 0; i < n[0]; ++i)
          A[(size_t)((k * n[1] + j) * n[0] + i) * m + col] = apply_L(&e, i, j, k);
  }
  grid_free(&e);
  for (int k = 0; k < n[2]; ++k)
    for (int j = 0; j < n[1]; ++j)
      for (int i = 0; i < n[0]; ++i) x[(k * n[1] + j) * n[0] + i] = get(rhs, i, j, k);
  for (int c = 0; c < m; ++c) {
    int best = c;
    for (int r = c + 1; r < m; ++r)
      if (fabs(A[(size_t)r * m + c]) > fabs(A[(size_t)best * m + c])) best = r;
    if (best != c) {
      for (int t = 0; t < m; ++t) {
        double tmp = A[(size_t)c * m + t];
        A[(size_t)c * m + t] = A[(size_t)best * m + t];
        A[(size_t)best * m + t] = tmp;
      }
      double tmp = x[c];
      x[c] = x[best];
      x[best] = tmp;
    }
    if (A[(size_t)c * m + c] == 0.0) die("singular coarse matrix");
    for (int r = c + 1; r < m; ++r) {
      double l = A[(size_t)r * m + c] / A[(size_t)c * m + c];
      for (int t = c + 1; t < m; ++t) A[(size_t)r * m + t] -= l * A[(size_t)c * m + t];
      x[r] -= l * x[c];
    }
  }
  for (int r = m - 1; r >= 0; --r) {
    double s = x[r];
    for (int t = r + 1; t < m; ++t) s -= A[(size_t)r * m + t] * x[t];
    x[r] = s / A[(size_t)r * m + r];
  }
  for (int k = 0; k < n[2]; ++k)
    for (int j = 0; j < n[1]; ++j)
      for (int i = 0; i < n[0]; ++i) put(u, i, j, k, x[(k * n[1] + j) * n[0] + i]);
  free(A);
  free(x);
}

/* ------------------------------------------------------------------------ */
/* global FAS V-cycle and FMG (Figs. 1 and 2)                                */
/* ------------------------------------------------------------------------ */

typedef struct {
  int pre, post, fmg; /* Chebyshev degrees: nu1, nu2, alpha */
} degrees;

typedef struct {
  int L;
  level *lv;
  grid *u, *rhs, *t, *res, *f;
} hierarchy;

static void level_of(level *lv, const int n[3], double h, int L, int l) {
  int s = L - 1 - l;
  for (int d = 0; d < 3; ++d) lv->n[d] = n[d] >> s;
  lv->h = h * (double)(1 << s);
}

static void hierarchy_new(hierarchy *H, const int n[3], double h, int L) {
  H->L = L;
  H->lv = (level *)calloc(L, sizeof(level));
  H->u = (grid *)calloc(L, sizeof(grid));
  H->rhs = (grid *)calloc(L, sizeof(grid));
  H->t = (grid *)calloc(L, sizeof(grid));
  H->res = (grid *)calloc(L, sizeof(grid));
  H->f = (grid *)calloc(L, sizeof(grid));
  if (!H->lv || !H->u || !H->rhs || !H->t || !H->res || !H->f) die("out of memory");
  for (int l = 0; l < L; ++l) {
    level_of(&H->lv[l], n, h, L, l);
    H->u[l] = grid_level(&H->lv[l]);
    H->rhs[l] = grid_level(&H->lv[l]);
    H->t[l] = grid_level(&H->lv[l]);
    H->res[l] = grid_level(&H->lv[l]);
    H->f[l] = grid_level(&H->lv[l]);
  }
}

static void hierarchy_free(hierarchy *H) {
  for (int l = 0; l < H->L; ++l) {
    grid_free(&H->u[l]);
    grid_free(&H->rhs[l]);
    grid_free(&H->t[l]);
    grid_free(&H->res[l]);
    grid_free(&H->f[l]);
  }
  free(H->lv);
  free(H->u);
  free(H->rhs);
  free(H->t);
  free(H->res);
  free(H->f);
}

/* FAS V-cycle on global level l with right-hand side *rhs (Fig. 1) */
static void fasmgv(hierarchy *H, int l, const grid *rhs, const degrees *dg) {
  grid *u = &H->u[l];
  region all = whole(u->n);
  if (l == 0) {
    coarse_solve(u, rhs);
    return;
  }
  cheb_smooth(u, rhs, &all, dg->pre);
  residual(&H->res[l], u, rhs, &all);
  grid *uc = &H->u[l - 1];
  const int *nc = uc->n;
#pragma omp parallel for schedule(static)
  for (int K = 0; K < nc[2]; ++K)
    for (int J = 0; J < nc[1]; ++J)
      for (int I = 0; I < nc[0]; ++I) put(uc, I, J, K, restrict_cell(u, I, J, K));
  copy_grid(&H->t[l - 1], uc);
#pragma omp parallel for schedule(static)
  for (int K = 0; K < nc[2]; ++K)
    for (int J = 0; J < nc[1]; ++J)
      for (int I = 0; I < nc[0]; ++I)
        put(&H->rhs[l - 1], I, J, K, restrict_cell(&H->res[l], I, J, K) + apply_L(uc, I, J, K));
  fasmgv(H, l - 1, &H->rhs[l - 1], dg);
  /* u += P(w - t), P trilinear: the coarse difference is formed first */
  grid *dc = &H->res[l - 1];
#pragma omp parallel for schedule(static)
  for (int K = 0; K < nc[2]; ++K)
    for (int J = 0; J < nc[1]; ++J)
      for (int I = 0; I < nc[0]; ++I)
        put(dc, I, J, K, get(uc, I, J, K) - get(&H->t[l - 1], I, J, K));
#pragma omp parallel for schedule(static)
  for (int k = 0; k < u->n[2]; ++k)
    for (int j = 0; j < u->n[1]; ++j)
      for (int i = 0; i < u->n[0]; ++i) put(u, i, j, k, get(u, i, j, k) + prolong_cell(dc, i, j, k));
  cheb_smooth(u, rhs, &all, dg->post);
}

static void load_f(hierarchy *H, const double *f) {
  int L = H->L;
  memcpy(H->f[L - 1].v, f, sizeof(double) * grid_count(&H->f[L - 1]));
  for (int l = L - 1; l > 0; --l) {
    grid *fc = &H->f[l - 1];
#pragma omp parallel for schedule(static)
    for (int K = 0; K < fc->n[2]; ++K)
      for (int J = 0; J < fc->n[1]; ++J)
        for (int I = 0; I < fc->n[0]; ++I) put(fc, I, J, K, restrict_cell(&H->f[l], I, J, K));
  }
}

static void prolong_global(grid *fine, const grid *coarse) {
#pragma omp parallel for schedule(static)
  for (int k = 0; k < fine->n[2]; ++k)
    for (int j = 0; j < fine->n[1]; ++j)
      for (int i = 0; i < fine->n[0]; ++i) put(fine, i, j, k, prolong_cell(coarse, i, j, k));
}

/* FMG stages 0..top on the global hierarchy (Fig. 2) */
static void fmg_global(hierarchy *H, int top, const degrees *dg) {
  coarse_solve(&H->u[0], &H->f[0]);
  for (int l = 1; l <= top; ++l) {
    region all = whole(H->u[l].n);
    prolong_global(&H->u[l], &H->u[l - 1]);
    cheb_smooth(&H->u[l], &H->f[l], &all, dg->fmg);
    fasmgv(H, l, &H->f[l], dg);
  }
}

/* ------------------------------------------------------------------------ */
/* segmental refinement (Sec. 4, Eq. 5, Figs. 5 and 6)                       */
/* ------------------------------------------------------------------------ */

typedef struct {
  int p[3];       /* segment coordinates */
  region V;       /* genuine region */
  region C;       /* compute region: V grown by J, clipped to the domain */
  grid u, rhs, t; /* storage over C plus one ghost layer */
} segment;

typedef struct {
  int L, K, T;
  int S[3];
  int *J;        /* J[l] for SR levels l = T+1..L-1, indexed by level */
  hierarchy G;   /* levels 0..L-1 as global arrays; SR levels use only f */
  segment **seg; /* seg[l][q] for l = T+1..L-1 */
} srstate;

static int nseg(const srstate *s) { return s->S[0] * s->S[1] * s->S[2]; }

static void seg_setup(segment *g, const level *lv, const int S[3], int Jl, int q) {
  int p[3] = {q % S[0], (q / S[0]) % S[1], q / (S[0] * S[1])};
  int lo[3], hi[3];
  for (int d = 0; d < 3; ++d) {
    int e = lv->n[d] / S[d];
    g->p[d] = p[d];
    g->V.a[d] = p[d] * e;
    g->V.b[d] = (p[d] + 1) * e;
    g->C.a[d] = g->V.a[d] - Jl < 0 ? 0 : g->V.a[d] - Jl;
    g->C.b[d] = g->V.b[d] + Jl > lv->n[d] ? lv->n[d] : g->V.b[d] + Jl;
    lo[d] = g->C.a[d] - 1;
    hi[d] = g->C.b[d] + 1;
  }
  g->u = grid_new(lv, lo, hi);
  g->rhs = grid_new(lv, lo, hi);
  g->t = grid_new(lv, lo, hi);
}

/* prolongation onto C u GSR of a segment grid (the storage cells inside the
 * domain) from source grid src: the FMG step when add == 0, the V-cycle
 * correction u += P(w - t) when add == 1 (src then holds w - t) */
static void sr_prolong(grid *u, const grid *src, int add) {
#pragma omp parallel for schedule(static)
  for (int c = 0; c < u->ext[2]; ++c)
    for (int b = 0; b < u->ext[1]; ++b)
      for (int a = 0; a < u->ext[0]; ++a) {
        int i = u->lo[0] + a, j = u->lo[1] + b, k = u->lo[2] + c;
        if (!in_domain(u->n, i, j, k)) continue;
        double v = prolong_cell(src, i, j, k);
        put(u, i, j, k, add ? get(u, i, j, k) + v : v);
      }
}

/* dst = w - t over the whole storage of w */
static void difference(grid *dst, const grid *w, const grid *t) {
  size_t cnt = grid_count(w);
  for (size_t c = 0; c < cnt; ++c) dst->v[c] = w->v[c] - t->v[c];
}

static const grid *sr_rhs(srstate *s, int l, int top, int q) {
  return (l == top) ? &s->G.f[l] : &s->seg[l][q].rhs;
}

/* per-segment part of Fig. 6 before the recursion on level l */
static void fasmgvsr_down(srstate *s, int l, int top, int q, const degrees *dg) {
  segment *g = &s->seg[l][q];
  const grid *rhs = sr_rhs(s, l, top, q);
  cheb_smooth(&g->u, rhs, &g->C, dg->pre);
  int hi[3] = {g->u.lo[0] + g->u.ext[0], g->u.lo[1] + g->u.ext[1], g->u.lo[2] + g->u.ext[2]};
  grid res = grid_new(&s->G.lv[l], g->u.lo, hi);
  residual(&res, &g->u, rhs, &g->C);
  if (l - 1 > s->T) {
    segment *c = &s->seg[l - 1][q];
    region F; /* F_{l-1} = C_l / 2 */
    for (int d = 0; d < 3; ++d) {
      F.a[d] = g->C.a[d] / 2;
      F.b[d] = g->C.b[d] / 2;
    }
    for (int K = F.a[2]; K < F.b[2]; ++K)
      for (int J = F.a[1]; J < F.b[1]; ++J)
        for (int I = F.a[0]; I < F.b[0]; ++I) put(&c->u, I, J, K, restrict_cell(&g->u, I, J, K));
    copy_grid(&c->t, &c->u);
    for (int K = c->C.a[2]; K < c->C.b[2]; ++K)
      for (int J = c->C.a[1]; J < c->C.b[1]; ++J)
        for (int I = c->C.a[0]; I < c->C.b[0]; ++I) {
          double Lu = apply_L(&c->u, I, J, K);
          double rr = in_region(&F, I, J, K) ? restrict_cell(&res, I, J, K) : 0.0;
          put(&c->rhs, I, J, K, rr + Lu);
        }
  } else {
    /* l - 1 = T: owner computes the genuine coarse cells of this segment */
    grid *uT = &s->G.u[s->T];
    grid *rT = &s->G.res[s->T];
    for (int K = g->V.a[2] / 2; K < g->V.b[2] / 2; ++K)
      for (int J = g->V.a[1] / 2; J < g->V.b[1] / 2; ++J)
        for (int I = g->V.a[0] / 2; I < g->V.b[0] / 2; ++I) {
          put(uT, I, J, K, restrict_cell(&g->u, I, J, K));
          put(rT, I, J, K, restrict_cell(&res, I, J, K));
        }
  }
  grid_free(&res);
}

static void fasmgvsr_up(srstate *s, int l, int top, int q, const degrees *dg) {
  segment *g = &s->seg[l][q];
  const grid *rhs = sr_rhs(s, l, top, q);
  if (l - 1 > s->T) {
    segment *c = &s->seg[l - 1][q];
    int hi[3] = {c->u.lo[0] + c->u.ext[0], c->u.lo[1] + c->u.ext[1], c->u.lo[2] + c->u.ext[2]};
    grid d = grid_new(&s->G.lv[l - 1], c->u.lo, hi);
    difference(&d, &c->u, &c->t);
    sr_prolong(&g->u, &d, 1);
    grid_free(&d);
  } else {
    sr_prolong(&g->u, &s->G.res[s->T], 1); /* holds w - t of the transition level */
  }
  cheb_smooth(&g->u, rhs, &g->C, dg->post);
}

/* FAS V-cycle with segmental refinement on SR level l (Fig. 6) */
static void fasmgvsr(srstate *s, int l, int top, const degrees *dg) {
  int ns = nseg(s);
#pragma omp parallel for schedule(dynamic)
  for (int q = 0; q < ns; ++q) fasmgvsr_down(s, l, top, q, dg);
  if (l - 1 > s->T) {
    fasmgvsr(s, l - 1, top, dg);
  } else {
    int T = s->T;
    hierarchy *H = &s->G;
    const int *n = H->u[T].n;
    copy_grid(&H->t[T], &H->u[T]);
#pragma omp parallel for schedule(static)
    for (int K = 0; K < n[2]; ++K)
      for (int J = 0; J < n[1]; ++J)
        for (int I = 0; I < n[0]; ++I)
          put(&H->rhs[T], I, J, K, get(&H->res[T], I, J, K) + apply_L(&H->u[T], I, J, K));
    fasmgv(H, T, &H->rhs[T], dg);
    /* w - t of the transition level, read by every segment's correction */
    difference(&H->res[T], &H->u[T], &H->t[T]);
  }
#pragma omp parallel for schedule(dynamic)
  for (int q = 0; q < ns; ++q) fasmgvsr_up(s, l, top, q, dg);
}

/* ------------------------------------------------------------------------ */
/* exported entry points                                                     */
/* ------------------------------------------------------------------------ */

/* levels: every extent divisible by 2^(L-1), coarsest extents <= 8 */
static int valid_levels(const int n[3], int L) {
  if (L < 1 || L > 30) return 0;
  int m = 1;
  for (int d = 0; d < 3; ++d) {
    if (n[d] < 1 || (n[d] >> (L - 1)) << (L - 1) != n[d]) return 0;
    int c = n[d] >> (L - 1);
    if (c > 8) return 0;
    m *= c;
  }
  return m <= 512;
}

static size_t count3(const int n[3]) { return (size_t)n[0] * n[1] * n[2]; }

/* out = L_h u on a whole grid of extents n and cell size h */
void orc27_apply(const double *u, const int *n, double h, double *out) {
  level lv = {{n[0], n[1], n[2]}, h};
  grid g = grid_level(&lv);
  memcpy(g.v, u, sizeof(double) * count3(n));
#pragma omp parallel for schedule(static)
  for (int k = 0; k < n[2]; ++k)
    for (int j = 0; j < n[1]; ++j)
      for (int i = 0; i < n[0]; ++i) out[((size_t)k * n[1] + j) * n[0] + i] = apply_L(&g, i, j, k);
  grid_free(&g);
}

/* degree-k Chebyshev smoothing of the whole grid, in place */
void orc27_cheb(double *u, const double *rhs, const int *n, double h, int degree) {
  level lv = {{n[0], n[1], n[2]}, h};
  grid g = grid_level(&lv), r = grid_level(&lv);
  memcpy(g.v, u, sizeof(double) * count3(n));
  memcpy(r.v, rhs, sizeof(double) * count3(n));
  region all = whole(n);
  cheb_smooth(&g, &r, &all, degree);
  memcpy(u, g.v, sizeof(double) * count3(n));
  grid_free(&g);
  grid_free(&r);
}

/* fine (2n) = trilinear prolongation of coarse (n) */
void orc27_prolong(const double *coarse, const int *n, double *fine) {
  level lc = {{n[0], n[1], n[2]}, 1.0}, lf = {{2 * n[0], 2 * n[1], 2 * n[2]}, 0.5};
  grid c = grid_level(&lc), f = grid_level(&lf);
  memcpy(c.v, coarse, sizeof(double) * count3(n));
  prolong_global(&f, &c);
  memcpy(fine, f.v, sizeof(double) * count3(lf.n));
  grid_free(&c);
  grid_free(&f);
}

/* u = A^{-1} rhs on a small grid (dense LU) */
int orc27_coarse_solve(const double *rhs, const int *n, double h, double *u) {
  if (count3(n) > 512) return -1;
  level lv = {{n[0], n[1], n[2]}, h};
  grid g = grid_level(&lv), r = grid_level(&lv);
  memcpy(r.v, rhs, sizeof(double) * count3(n));
  coarse_solve(&g, &r);
  memcpy(u, g.v, sizeof(double) * count3(n));
  grid_free(&g);
  grid_free(&r);
  return 0;
}

/* Global FMG (Fig. 2): f, u with extents n (x fastest), finest cell size h */
int orc27_fmg(const double *f, const int *n, double h, int L, int pre, int post, int fmgdeg,
              double *u) {
  if (!valid_levels(n, L) || pre < 0 || post < 0 || fmgdeg < 0) return -1;
  degrees dg = {pre, post, fmgdeg};
  hierarchy H;
  hierarchy_new(&H, n, h, L);
  load_f(&H, f);
  fmg_global(&H, L - 1, &dg);
  memcpy(u, H.u[L - 1].v, sizeof(double) * count3(n));
  hierarchy_free(&H);
  return 0;
}

/* Iterated global FAS V-cycles from the guess in u until
 * max|f - L u| <= rtol max|f| or maxit cycles; returns the cycle count and
 * the final relative residual in *relres. */
int orc27_vcycles(const double *f, const int *n, double h, int L, int pre, int post,
                  double rtol, int maxit, double *u, double *relres) {
  if (!valid_levels(n, L)) return -1;
  degrees dg = {pre, post, 0};
  hierarchy H;
  hierarchy_new(&H, n, h, L);
  load_f(&H, f);
  memcpy(H.u[L - 1].v, u, sizeof(double) * count3(n));
  region all = whole(n);
  double fn = 0.0;
  for (size_t c = 0; c < count3(n); ++c) fn = fmax(fn, fabs(f[c]));
  int it = 0;
  double rn = 0.0;
  for (;;) {
    residual(&H.res[L - 1], &H.u[L - 1], &H.f[L - 1], &all);
    rn = 0.0;
    for (size_t c = 0; c < count3(n); ++c) rn = fmax(rn, fabs(H.res[L - 1].v[c]));
    if (rn <= rtol * fn || it >= maxit) break;
    fasmgv(&H, L - 1, &H.f[L - 1], &dg);
    ++it;
  }
  memcpy(u, H.u[L - 1].v, sizeof(double) * count3(n));
  hierarchy_free(&H);
  if (relres) *relres = fn > 0 ? rn / fn : rn;
  return it;
}

/* FMG with segmental refinement on the K finest levels (Figs. 5 and 6).
 * S: segments per dimension (each extent divisible by S[d] * 2^K, genuine
 * regions cubic); J: K buffer widths, finest level first, each even and at
 * least half the next finer one. */
int orc27_srfmg(const double *f, const int *n, double h, int L, int K, const int *S, const int *J,
                int pre, int post, int fmgdeg, double *u) {
  if (!valid_levels(n, L) || K < 0 || K > L - 1 || pre < 0 || post < 0 || fmgdeg < 0) return -1;
  if (K == 0) return orc27_fmg(f, n, h, L, pre, post, fmgdeg, u);
  for (int d = 0; d < 3; ++d)
    if (S[d] < 1 || n[d] % (S[d] << K) != 0) return -1;
  if (n[0] / S[0] != n[1] / S[1] || n[0] / S[0] != n[2] / S[2]) return -1;
  for (int i = 0; i < K; ++i) {
    if (J[i] < 0 || (J[i] & 1)) return -1;
    if (i + 1 < K && 2 * J[i + 1] < J[i]) return -1;
  }
  degrees dg = {pre, post, fmgdeg};
  srstate s;
  s.L = L;
  s.K = K;
  s.T = L - 1 - K;
  for (int d = 0; d < 3; ++d) s.S[d] = S[d];
  s.J = (int *)calloc(L, sizeof(int));
  s.seg = (segment **)calloc(L, sizeof(segment *));
  if (!s.J || !s.seg) die("out of memory");
  hierarchy_new(&s.G, n, h, L);
  load_f(&s.G, f);
  int ns = nseg(&s);
  for (int l = s.T + 1; l < L; ++l) {
    s.J[l] = J[L - 1 - l];
    s.seg[l] = (segment *)calloc(ns, sizeof(segment));
    if (!s.seg[l]) die("out of memory");
    for (int q = 0; q < ns; ++q) seg_setup(&s.seg[l][q], &s.G.lv[l], S, s.J[l], q);
  }
  /* global FMG up to the transition level */
  fmg_global(&s.G, s.T, &dg);
  /* w - t is zero until the first V-cycle below forms it */
  for (int top = s.T + 1; top < L; ++top) {
#pragma omp parallel for schedule(dynamic)
    for (int q = 0; q < ns; ++q) {
      segment *g = &s.seg[top][q];
      const grid *src = (top - 1 == s.T) ? &s.G.u[s.T] : &s.seg[top - 1][q].u;
      sr_prolong(&g->u, src, 0);
      cheb_smooth(&g->u, &s.G.f[top], &g->C, dg.fmg);
    }
    fasmgvsr(&s, top, top, &dg);
  }
  /* output: genuine cells of the finest segments */
  for (int q = 0; q < ns; ++q) {
    segment *g = &s.seg[L - 1][q];
    for (int k = g->V.a[2]; k < g->V.b[2]; ++k)
      for (int j = g->V.a[1]; j < g->V.b[1]; ++j)
        for (int i = g->V.a[0]; i < g->V.b[0]; ++i)
          u[((size_t)k * n[1] + j) * n[0] + i] = get(&g->u, i, j, k);
  }
  for (int l = s.T + 1; l < L; ++l) {
    for (int q = 0; q < ns; ++q) {
      grid_free(&s.seg[l][q].u);
      grid_free(&s.seg[l][q].rhs);
      grid_free(&s.seg[l][q].t);
    }
    free(s.seg[l]);
  }
  hierarchy_free(&s.G);
  free(s.seg);
  free(s.J);
  return 0;
}

int orc27_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
