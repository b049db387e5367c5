// kernels_coarse.hpp -- the coarse global levels in one persistent workgroup.
//
// Levels whose grids are small (up to 16^3 cells) are latency bound: a kernel
// launch per operator costs more than the work.  k_coarse runs every
// operator of these levels inside one workgroup, with a block barrier between
// phases, on copies of the levels held in LDS: it loads what the cycle reads
// (the top level's u and right-hand side, or the FMG right-hand sides), works
// in LDS and writes back the top level's u, the only result used outside.
// It performs either
//   mode 0: FMG stages 0..top (Fig. 2 of the paper): f_top is restricted
//           down to level 0, u_0 = L_0^-1 f_0, then per level Pi, S^alpha and
//           one FAS V-cycle with rhs f_l, or
//   mode 1: one FAS V-cycle (Fig. 1) on level top with right-hand side rt;
//           with fas, rt holds the restricted residual of the level above and
//           the kernel first forms the FAS right-hand side rt + L u (Eq. 4)
//           and stores t = u, the values the coarse-grid correction subtracts.
//
// LDS layout: each level's u is stored with a one-cell halo of zeros
// ((n+2)^3 elements), so a 7-point sum reads its six neighbours without
// bounds tests (a zero stands for the eliminated Dirichlet ghost; the
// diagonal 6 + nb carries the boundary).  t, the right-hand sides and f are
// read point-wise and stored unpadded (n^3, x fastest).  The host forms the
// offsets (coarse_layout); a small coarsest inverse is staged in LDS too.
//
// With 16 wavefronts on the 4 SIMDs of one CU, every vector instruction a
// thread issues costs ~16 cycles of the phase, so the phases keep per-thread
// index arithmetic small: divisions by level extents use the reciprocal
// (udiv_small), the smoother and the 16^3 correction and FAS right-hand side
// are also compiled for constant edges (immediate LDS offsets), each
// thread's smoother cells and right-hand sides are set up once per call, and
// the restriction and correction spread their work over all threads.  Each
// operator is inlined once (a single loop over the steps of the cycle), which
// keeps the kernel's code within reach of the instruction cache.
#pragma once
#include <type_traits>
#include "grid.hpp"
#include "kernels_simple.hpp"

namespace fmg {

constexpr int kCoarseMaxLevels = 8;
constexpr int kCoarseThreads = 1024;
constexpr int kCoarseAinvLds = 32;  // coarsest levels of up to 32 cells keep A^-1 in LDS

template <class T>
struct CoarseArgs {
  T* u[kCoarseMaxLevels];
  T* t[kCoarseMaxLevels];
  T* r[kCoarseMaxLevels];        // rhs of the V-cycle on each level below top
  const T* f[kCoarseMaxLevels];  // FMG right-hand sides
  int n[kCoarseMaxLevels];
  const double* Ainv;
  int mm;
  int top;
  int mode;
  const T* rt;  // mode 1: rhs of level top (with fas: R res of the level above)
  int fas;      // mode 1: form the FAS right-hand side rt + L u and t = u of level top
  int nu1, nu2, alpha;
  double* ck[kCoarseMaxLevels];  // mode 0: level l's solution after its stage (or null)
  // LDS layout (coarse_layout), in elements of T: padded u, t and the V-cycle
  // rhs of each level, f (mode 0), the top level's rhs (mode 1); A^-1 at byte
  // offset oai, or oai = -1 when it is read from global memory
  int ou[kCoarseMaxLevels], ot[kCoarseMaxLevels], orh[kCoarseMaxLevels], of[kCoarseMaxLevels];
  int ort, oai;
};

// elements of a level's padded u
__host__ __device__ inline int coarse_padded(int n) {
  const int p = n + 2;
  return p * p * p;
}

// The LDS layout of k_coarse for levels 0..top with edges n: the u of every
// level, then t and rhs of the levels below top, f of every level (mode 0),
// the top level's rhs (mode 1), and the coarsest inverse (mm cells, FP64,
// 8-byte aligned) when mm <= kCoarseAinvLds.  Offsets go to the arrays given
// (any may be null); returns the bytes needed for elements of esz bytes.
inline size_t coarse_layout(const int* n, int top, int mode, int mm, size_t esz, int* ou = nullptr,
                            int* ot = nullptr, int* orh = nullptr, int* of = nullptr,
                            int* ort = nullptr, int* oai = nullptr) {
  int off = 0;
  for (int l = 0; l <= top; ++l) {
    if (ou) ou[l] = off;
    off += coarse_padded(n[l]);
  }
  for (int l = 0; l <= top; ++l) {
    const int c = n[l] * n[l] * n[l];
    if (ot) ot[l] = 0;
    if (orh) orh[l] = 0;
    if (l < top) {
      if (ot) ot[l] = off;
      off += c;
      if (orh) orh[l] = off;
      off += c;
    }
  }
  for (int l = 0; l <= top; ++l) {
    if (of) of[l] = 0;
    if (mode == 0) {
      if (of) of[l] = off;
      off += n[l] * n[l] * n[l];
    }
  }
  if (ort) *ort = off;
  if (mode == 1) off += n[top] * n[top] * n[top];
  size_t bytes = esz * (size_t)off;
  if (oai) *oai = -1;
  if (mm <= kCoarseAinvLds) {
    bytes = (bytes + 7) & ~(size_t)7;
    if (oai) *oai = (int)bytes;
    bytes += sizeof(double) * (size_t)mm * (size_t)mm;
  }
  return bytes;
}

// padded index of cell (x, y, z) of an n^3 level
__device__ inline int pidx(int n, int x, int y, int z) {
  const int p = n + 2;
  return ((z + 1) * p + (y + 1)) * p + (x + 1);
}

// cell (i, j, k) of an ex x ey x * box walked from linear index c0 in strides
// of `stride` (the grid-wide Walk3 with the small-operand division)
struct CWalk {
  int i, j, k, di, dj, dk, ex, ey;
  __device__ CWalk(int c0, int stride, int ex_, int ey_) : ex(ex_), ey(ey_) {
    const int exy = ex * ey;
    k = udiv_small(c0, exy);
    const int r = c0 - k * exy;
    j = udiv_small(r, ex);
    i = r - j * ex;
    dk = udiv_small(stride, exy);
    const int rs = stride - dk * exy;
    dj = udiv_small(rs, ex);
    di = rs - dj * ex;
  }
  __device__ void next() {
    i += di;
    j += dj;
    k += dk;
    if (i >= ex) {
      i -= ex;
      ++j;
    }
    if (j >= ey) {
      j -= ey;
      ++k;
    }
  }
};

// threadIdx.x hidden from the optimizer: the per-thread setup of a phase
// depends only on it and on level constants, and would otherwise be hoisted
// out of the loop over steps and held in registers across the whole cycle
__device__ inline int opaque_tid() {
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

// the value of lane ^ 1 (DPP quad permutation 1, 0, 3, 2)
__device__ inline double lane_swap1(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0xB1, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0xB1, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// 1 / (6 + nb) for nb = 0..6 boundary faces (constants, no division)
template <class T>
__device__ inline T inv_diag(int nb) {
  T r = (T)(1.0 / 6.0);
  r = nb == 1 ? (T)(1.0 / 7.0) : r;
  r = nb == 2 ? (T)(1.0 / 8.0) : r;
  r = nb == 3 ? (T)(1.0 / 9.0) : r;
  r = nb == 4 ? (T)(1.0 / 10.0) : r;
  r = nb == 5 ? (T)(1.0 / 11.0) : r;
  r = nb == 6 ? (T)(1.0 / 12.0) : r;
  return r;
}

// one cell of each colour: the i-th cell of colour 0 and its x-neighbour,
// which is the i-th cell of colour 1 (n is even).  Cells are numbered x
// fastest within pairs of rows (y, y + 1), alternating between the two rows:
// a row's cells of one colour lie two apart, and the checkerboard shifts
// them by one between the rows, so alternating lanes fall on the other half
// of the LDS banks (two rows apart by 2(n + 2) + -2 words, 2 mod 4) and a
// wavefront's 64-bit reads use every bank equally.
template <class T>
struct GsCell {
  int p, c, d;  // padded and plain index of the colour-0 cell; colour-1 offset
  T inv0, inv1;
  bool v;
};

template <class T>
__device__ inline GsCell<T> gs_cell(int i, int n, int half) {
  GsCell<T> g;
  g.v = i < half;
  // idle slots point at cell (0,0,0), read valid cells and store nothing;
  // wavefronts without a cell of this level skip the index arithmetic
  g.p = pidx(n, 0, 0, 0);
  g.c = 0;
  g.d = 1;
  g.inv0 = g.inv1 = (T)0;
  if (g.v) {
    const int hx = n >> 1;
    const int rp = udiv_small(i, 2 * hx), w = i - rp * 2 * hx;  // pair of rows, place in it
    const int row = 2 * rp + (w & 1), xh = w >> 1;
    const int z = udiv_small(row, n), y = row - z * n;
    const int q = (y + z) & 1;
    const int x0 = 2 * xh + q, x1 = 2 * xh + 1 - q;
    g.p = pidx(n, x0, y, z);
    g.c = (z * n + y) * n + x0;
    g.d = x1 - x0;
    const int nyz = (y == 0) + (y == n - 1) + (z == 0) + (z == n - 1);
    g.inv0 = inv_diag<T>(nyz + (x0 == 0) + (x0 == n - 1));
    g.inv1 = inv_diag<T>(nyz + (x1 == 0) + (x1 == n - 1));
  }
  return g;
}

// Gauss-Seidel update of the cell at padded index p with right-hand side r
template <class T>
__device__ inline T gs_value(const T* u, int p, int P, int P2, T h2, T r, T inv) {
  const T s = ((u[p - 1] + u[p + 1]) + (u[p - P] + u[p + P])) + (u[p - P2] + u[p + P2]);
  return (s - h2 * r) * inv;
}

// nu red-black sweeps in place, red ((x + y + z) even) first; u padded.
// Each thread owns up to two cells per colour (edges up to 16: at most
// 2 kCoarseThreads cells per colour); their indices, diagonals and
// right-hand sides are set up once for the nu sweeps.  NE: the edge as a
// constant (16), or 0.
template <class T, int NE>
__device__ void blk_gs(T* u, const T* rhs, int n_, int nu) {
  if (nu <= 0) return;
  constexpr int NT = kCoarseThreads;
  const int n = NE ? NE : n_;
  const double h = 1.0 / (double)n;
  const T h2 = (T)(h * h);
  const int P = n + 2, P2 = P * P, half = n * n * (n >> 1);
  const int t = opaque_tid();
  const GsCell<T> a = gs_cell<T>(t, n, half), b = gs_cell<T>(t + NT, n, half);
  const T ra0 = rhs[a.c], ra1 = rhs[a.c + a.d], rb0 = rhs[b.c], rb1 = rhs[b.c + b.d];
  const bool two = half > NT;  // uniform
  for (int it = 0; it < nu; ++it)
    for (int col = 0; col < 2; ++col) {
      if (a.v) {  // loads of both cells before the stores
        const int pa = a.p + (col ? a.d : 0), pb = b.p + (col ? b.d : 0);
        const T va = gs_value(u, pa, P, P2, h2, col ? ra1 : ra0, col ? a.inv1 : a.inv0);
        if (two) {
          const T vb = gs_value(u, pb, P, P2, h2, col ? rb1 : rb0, col ? b.inv1 : b.inv0);
          u[pa] = va;
          if (b.v) u[pb] = vb;
        } else {
          u[pa] = va;
        }
      }
      __syncthreads();
    }
}

// uc = R u, rc = R (rhs - L u) on every coarse cell; then t = uc and
// rc = rc + L_H uc (FAS right-hand side, Eq. 4).  u, uc padded.  Two
// neighbouring lanes take one coarse cell: each the four children of one of
// its two fine planes, reading the 2 x 2 block and its 16 face neighbours
// once; the two halves are added across the lane pair.
template <class T>
__device__ void blk_descend(const T* u, const T* rhs, int n, T* uc, T* rc, T* tc) {
  constexpr int NT = kCoarseThreads;
  const int nc = n / 2, cc = nc * nc * nc;
  const int P = n + 2, P2 = P * P;
  const double s2 = (double)n * (double)n;
  const int tid = opaque_tid(), hz = tid & 1;
  CWalk w(tid >> 1, NT >> 1, nc, nc);  // (I, J, K) of coarse cell c
#pragma unroll 1
  for (int c = tid >> 1; c < cc; c += NT >> 1, w.next()) {
    const int x0 = 2 * w.i, y0 = 2 * w.j, z = 2 * w.k + hz;
    const int p = pidx(n, x0, y0, z);  // child (0, 0) of this plane
    double b[2][2], xm[2], xp[2], ym[2], yp[2], zm[2][2], zp[2][2];
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        b[j][i] = (double)u[p + j * P + i];
        zm[j][i] = (double)u[p + j * P + i - P2];
        zp[j][i] = (double)u[p + j * P + i + P2];
      }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      xm[q] = (double)u[p + q * P - 1];
      xp[q] = (double)u[p + q * P + 2];
      ym[q] = (double)u[p + q - P];
      yp[q] = (double)u[p + q + 2 * P];
    }
    const int nz = (z == 0) + (z == n - 1);
    double su = 0.0, sr = 0.0;
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int x = x0 + i, y = y0 + j;
        const double v = b[j][i];
        const double s = ((i ? b[j][0] : xm[j]) + (i ? xp[j] : b[j][1])) +
                         ((j ? b[0][i] : ym[i]) + (j ? yp[i] : b[1][i])) + (zm[j][i] + zp[j][i]);
        const int nb = (x == 0) + (x == n - 1) + (y == 0) + (y == n - 1) + nz;
        su += v;
        sr += (double)rhs[(z * n + y) * n + x] - (s - (double)(6 + nb) * v) * s2;
      }
    // the lane pair of c is active together (c is the same for both)
    su += lane_swap1(su);
    sr += lane_swap1(sr);
    if (hz == 0) {
      uc[pidx(nc, w.i, w.j, w.k)] = (T)(su / 8.0);
      rc[c] = (T)(sr / 8.0);
    }
  }
  __syncthreads();
  const int Pc = nc + 2, Pc2 = Pc * Pc;
  const double sc2 = (double)nc * (double)nc;
  CWalk w2(tid, NT, nc, nc);
#pragma unroll 1
  for (int c = tid; c < cc; c += NT, w2.next()) {
    const int K = w2.k, J = w2.j, I = w2.i;
    const int p = pidx(nc, I, J, K);
    const double v = (double)uc[p];
    const double s = (((double)uc[p - 1] + (double)uc[p + 1]) +
                      ((double)uc[p - Pc] + (double)uc[p + Pc])) +
                     ((double)uc[p - Pc2] + (double)uc[p + Pc2]);
    const int nb = (I == 0) + (I == nc - 1) + (J == 0) + (J == nc - 1) + (K == 0) + (K == nc - 1);
    tc[c] = uc[p];
    rc[c] = (T)((double)rc[c] + (s - (double)(6 + nb) * v) * sc2);
  }
  __syncthreads();
}

// u += P(w - t): each fine cell adds the increment of its coarse parent;
// u and w padded, t plain
template <class T, int NE>
__device__ void blk_correct(T* u, int n_, const T* w, const T* t) {
  constexpr int NT = kCoarseThreads;
  const int n = NE ? NE : n_;
  const int nc = n / 2, cnt = n * n * n;
  const int tid = opaque_tid();
  CWalk wk(tid, NT, n, n);
#pragma unroll 1
  for (int i = tid; i < cnt; i += NT, wk.next()) {
    const int x = wk.i, y = wk.j, z = wk.k, X = x >> 1, Y = y >> 1, Z = z >> 1;
    const T d = w[pidx(nc, X, Y, Z)] - t[(Z * nc + Y) * nc + X];
    const int p = pidx(n, x, y, z);
    u[p] = (T)(u[p] + d);
  }
  __syncthreads();
}

// FMG interpolation Pi (trilinear, odd reflection at the boundary) of the
// padded coarse c onto the padded fine u.  Per axis a fine cell takes 3/4 of
// its parent's coarse plane and 1/4 of the next one on its side; beyond a
// wall that one is the parent itself, entering with sign -1.
template <class T>
__device__ void blk_interp(T* u, int n, const T* c) {
  constexpr int NT = kCoarseThreads;
  const int cnt = n * n * n, nc = n / 2, Pc = nc + 2, Pc2 = Pc * Pc;
  const T* c0 = c + pidx(nc, 0, 0, 0);
  const int tid = opaque_tid();
  CWalk w(tid, NT, n, n);
#pragma unroll 1
  for (int i = tid; i < cnt; i += NT, w.next()) {
    const int f[3] = {w.i, w.j, w.k};
    int near[3], far[3];
    bool neg[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int p = f[d] >> 1, r = (f[d] & 1) ? p + 1 : p - 1;
      neg[d] = r < 0 || r >= nc;
      near[d] = p;
      far[d] = neg[d] ? p : r;
    }
    T s = 0;
#pragma unroll
    for (int cz = 0; cz < 2; ++cz)
#pragma unroll
      for (int cy = 0; cy < 2; ++cy)
#pragma unroll
        for (int cx = 0; cx < 2; ++cx) {
          const T wt = (T)((cx ? 0.25 : 0.75) * (cy ? 0.25 : 0.75) * (cz ? 0.25 : 0.75));
          const bool ng = (cx && neg[0]) != ((cy && neg[1]) != (cz && neg[2]));
          const T sign = ng ? (T)-1 : (T)1;
          const int o = (cz ? far[2] : near[2]) * Pc2 + (cy ? far[1] : near[1]) * Pc +
                        (cx ? far[0] : near[0]);
          s += wt * sign * c0[o];
        }
    u[pidx(n, w.i, w.j, w.k)] = s;
  }
  __syncthreads();
}

// exact coarsest solve u0 = A^-1 rhs0 (rhs0 plain, u0 padded); A in LDS or
// global memory
template <class T>
__device__ void blk_coarse_solve(T* u0, const T* rhs0, int n0, const double* A, int mm) {
  for (int r = threadIdx.x; r < mm; r += blockDim.x) {
    double s = 0.0;
#pragma unroll 8
    for (int c = 0; c < mm; ++c) s += A[r * mm + c] * (double)rhs0[c];
    const int z = udiv_small(r, n0 * n0), rr = r - z * n0 * n0, y = udiv_small(rr, n0);
    u0[pidx(n0, rr - y * n0, y, z)] = (T)s;
  }
  __syncthreads();
}

template <class T>
__device__ void coarse_solve(unsigned char* raw, T* sm, const CoarseArgs<T>& g, int rofs) {
  if (g.oai >= 0)
    blk_coarse_solve(sm + g.ou[0], sm + rofs, g.n[0],
                     reinterpret_cast<const double*>(raw + g.oai), g.mm);
  else
    blk_coarse_solve(sm + g.ou[0], sm + rofs, g.n[0], g.Ainv, g.mm);
}

// FAS right-hand side of the top level in LDS: r += L u (Eq. 2, in FP64) on
// every cell; u padded, r plain (t = u was stored by the first phase)
template <class T, int NE>
__device__ void blk_fas_rhs(const T* u, T* r, int n_) {
  constexpr int NT = kCoarseThreads;
  const int n = NE ? NE : n_;
  const int cnt = n * n * n, P = n + 2, P2 = P * P;
  const double s2 = (double)n * (double)n;
  const int tid = opaque_tid();
  CWalk w(tid, NT, n, n);
#pragma unroll 1
  for (int c = tid; c < cnt; c += NT, w.next()) {
    const int x = w.i, y = w.j, z = w.k;
    const int p = pidx(n, x, y, z);
    const double v = (double)u[p];
    const double s = (((double)u[p - 1] + (double)u[p + 1]) + ((double)u[p - P] + (double)u[p + P])) +
                     ((double)u[p - P2] + (double)u[p + P2]);
    const int nb = (x == 0) + (x == n - 1) + (y == 0) + (y == n - 1) + (z == 0) + (z == n - 1);
    r[c] = (T)((double)r[c] + (s - (double)(6 + nb) * v) * s2);
  }
  __syncthreads();
}

// The first phase: loads of the top level's data (mode 0: f; mode 1: rhs and
// u) are issued first; while they are in flight the halos are zeroed (every
// padded u below the top level whole, the top level's halo cell by cell)
// and a small A^-1 is staged; then the loaded values are stored (with fas
// also t = u of the top level, straight from the loaded registers).
template <class T>
__device__ void blk_start(unsigned char* raw, T* sm, const CoarseArgs<T>& g) {
  constexpr int NT = kCoarseThreads;
  const int top = g.top, n = g.n[top], cnt = n * n * n;
  const int P = n + 2;
  const bool m1 = g.mode == 1, fas = m1 && g.fas;
  const T* src = m1 ? g.rt : g.f[top];
  T* dst = sm + (m1 ? g.ort : g.of[top]);
  T* ut = sm + g.ou[top];
  const T* gu = g.u[top];
  T* gt = g.t[top];
  const int tid = opaque_tid();
  CWalk w(tid, NT, n, n);
#pragma unroll 1
  for (int base = 0; base < cnt; base += 4 * NT) {
    T v1[4], v2[4];
    int li[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int i = base + tid + k * NT;
      const bool in = i < cnt;
      li[k] = in ? pidx(n, w.i, w.j, w.k) : 0;
      w.next();
      v1[k] = in ? src[i] : (T)0;
      v2[k] = (in && m1) ? gu[i] : (T)0;
    }
    if (base == 0) {
#pragma unroll 1
      for (int i = tid; i < g.ou[top]; i += NT) sm[i] = (T)0;
      // top halo: the planes z = 0 and z = P - 1, then rows y = 0 and
      // y = P - 1 of the inner planes, then cells x = 0 and x = P - 1 of the
      // inner rows
      const int H1 = 2 * P * P, H2 = H1 + 2 * n * P, H3 = H2 + 2 * n * n;
#pragma unroll 1
      for (int k = tid; k < H3; k += NT) {
        int e;
        if (k < H1) {
          e = k < P * P ? k : (P - 1) * P * P + (k - P * P);
        } else if (k < H2) {
          const int q = k - H1, z = udiv_small(q, 2 * P), r = q - z * 2 * P;
          e = ((z + 1) * P + (r < P ? 0 : P - 1)) * P + (r < P ? r : r - P);
        } else {
          const int q = k - H2, row = q >> 1, z = udiv_small(row, n), y = row - z * n;
          e = ((z + 1) * P + (y + 1)) * P + ((q & 1) ? P - 1 : 0);
        }
        ut[e] = (T)0;
      }
      if (g.oai >= 0) {
        double* ai = reinterpret_cast<double*>(raw + g.oai);
#pragma unroll 1
        for (int k = tid; k < g.mm * g.mm; k += NT) ai[k] = g.Ainv[k];
      }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int i = base + tid + k * NT;
      if (i < cnt) {
        dst[i] = v1[k];
        if (m1) ut[li[k]] = v2[k];
        if (fas) gt[i] = v2[k];
      }
    }
  }
  __syncthreads();
}

// the top level's u (padded LDS) back to global memory
template <class T>
__device__ void blk_store_top(const T* lds, T* glob, int n) {
  constexpr int NT = kCoarseThreads;
  const int cnt = n * n * n;
  const int tid = opaque_tid();
  CWalk w(tid, NT, n, n);
#pragma unroll 1
  for (int i = tid; i < cnt; i += NT, w.next()) glob[i] = lds[pidx(n, w.i, w.j, w.k)];
}

// f of level l - 1 = R f of level l (mean of the 8 children, summed in FP64
// in the order of the global restriction kernel); both plain, in LDS
template <class T>
__device__ void blk_restrict_f(const T* f, int n, T* fc) {
  constexpr int NT = kCoarseThreads;
  const int nc = n / 2, cnt = nc * nc * nc;
  const int tid = opaque_tid();
  CWalk w(tid, NT, nc, nc);
#pragma unroll 1
  for (int c = tid; c < cnt; c += NT, w.next()) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int i = 0; i < 2; ++i)
          s += (double)f[((2 * w.k + k) * n + (2 * w.j + j)) * n + (2 * w.i + i)];
    fc[c] = (T)(s / 8.0);
  }
  __syncthreads();
}

// a level's solution (padded LDS) to an FP64 checkpoint array (n^3)
template <class T>
__device__ void blk_checkpoint(const T* lds, double* out, int n) {
  const int cnt = n * n * n;
  const int tid = opaque_tid();
  CWalk w(tid, kCoarseThreads, n, n);
#pragma unroll 1
  for (int i = tid; i < cnt; i += kCoarseThreads, w.next())
    out[i] = (double)lds[pidx(n, w.i, w.j, w.k)];
}

// The kernel walks one sequence of steps, so that each operator is
// instantiated once (the code of a cycle is fetched once per launch, and the
// instruction cache is shared by two CUs).  Stage lt is an FMG stage (mode 0:
// lt = 1..top) or the V-cycle (mode 1: lt = top); its steps s are
//   s = -1 (mode 0): Pi onto level lt, then S^alpha with f_lt;
//   s = 0..lt-1:     S^nu1 on level lt - s, then restriction (descent);
//   s = lt:          the exact coarsest solve;
//   s = lt+1..2 lt:  correction of level s - lt, then S^nu2 (ascent).
// The smoother, whose phases repeat, is also instantiated for edges 16 and 8.
template <class T>
__global__ void __launch_bounds__(kCoarseThreads) k_coarse(CoarseArgs<T> g) {
  extern __shared__ unsigned char smem_raw[];  // offset 0: no static LDS
  T* sm = reinterpret_cast<T*>(smem_raw);
  const int top = g.top;
  const bool m0 = g.mode == 0;
  blk_start(smem_raw, sm, g);
  if (m0) {
#pragma unroll 1
    for (int l = top; l >= 1; --l) blk_restrict_f(sm + g.of[l], g.n[l], sm + g.of[l - 1]);
    coarse_solve(smem_raw, sm, g, g.of[0]);
    if (g.ck[0]) blk_checkpoint(sm + g.ou[0], g.ck[0], g.n[0]);
  } else if (g.fas) {
    if (g.n[top] == 16) blk_fas_rhs<T, 16>(sm + g.ou[top], sm + g.ort, g.n[top]);
    else blk_fas_rhs<T, 0>(sm + g.ou[top], sm + g.ort, g.n[top]);
  }
#pragma unroll 1
  for (int lt = m0 ? 1 : top; lt <= top; ++lt) {
    const int rto = m0 ? g.of[lt] : g.ort;  // rhs of level lt
#pragma unroll 1
    for (int s = m0 ? -1 : 0; s <= 2 * lt; ++s) {
      if (s == lt) {
        coarse_solve(smem_raw, sm, g, lt == 0 ? rto : g.orh[0]);
        continue;
      }
      const int l = s < 0 ? lt : s < lt ? lt - s : s - lt;
      const int n = g.n[l];
      T* ul = sm + g.ou[l];
      T* rhs = sm + (l == lt ? rto : g.orh[l]);
      if (s < 0) blk_interp(ul, n, sm + g.ou[l - 1]);
      if (s > lt) {
        if (n == 16) blk_correct<T, 16>(ul, n, sm + g.ou[l - 1], sm + g.ot[l - 1]);
        else if (n == 8) blk_correct<T, 8>(ul, n, sm + g.ou[l - 1], sm + g.ot[l - 1]);
        else blk_correct<T, 0>(ul, n, sm + g.ou[l - 1], sm + g.ot[l - 1]);
      }
      const int nu = s < 0 ? g.alpha : s < lt ? g.nu1 : g.nu2;
      if (n == 16) blk_gs<T, 16>(ul, rhs, n, nu);
      else if (n == 8) blk_gs<T, 8>(ul, rhs, n, nu);
      else if (n == 4) blk_gs<T, 4>(ul, rhs, n, nu);
      else blk_gs<T, 0>(ul, rhs, n, nu);
      if (s >= 0 && s < lt)
        blk_descend(ul, rhs, n, sm + g.ou[l - 1], sm + g.orh[l - 1], sm + g.ot[l - 1]);
    }
    if (m0 && g.ck[lt]) blk_checkpoint(sm + g.ou[lt], g.ck[lt], g.n[lt]);
  }
  blk_store_top(sm + g.ou[top], g.u[top], g.n[top]);
}

}  // namespace fmg
