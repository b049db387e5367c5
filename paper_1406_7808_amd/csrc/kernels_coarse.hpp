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
// read point-wise and stored unpadded (n^3, x fastest).  Threads are mapped
// to the cells of one colour, so every thread of a half-sweep has work and
// all its loads are issued before its stores.
#pragma once
#include "grid.hpp"
#include "kernels_simple.hpp"

namespace fmg {

constexpr int kCoarseMaxLevels = 8;
constexpr int kCoarseThreads = 1024;

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
};

// elements of a level's padded u
__host__ __device__ inline int coarse_padded(int n) {
  const int p = n + 2;
  return p * p * p;
}

// padded index of cell (x, y, z) of an n^3 level
__device__ inline int pidx(int n, int x, int y, int z) {
  const int p = n + 2;
  return ((z + 1) * p + (y + 1)) * p + (x + 1);
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
    const int rp = i / (2 * hx), w = i - rp * 2 * hx;  // pair of rows, place in it
    const int row = 2 * rp + (w & 1), xh = w >> 1;
    const int z = row / n, y = row - z * n;
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

// Gauss-Seidel update of two cells of colour col: loads, then stores
template <class T>
__device__ inline void gs_pair(T* u, const T* rhs, int P, int P2, T h2, int col,
                               const GsCell<T>& a, const GsCell<T>& b) {
  const int pa = a.p + (col ? a.d : 0), ca = a.c + (col ? a.d : 0);
  const int pb = b.p + (col ? b.d : 0), cb = b.c + (col ? b.d : 0);
  const T sa = ((u[pa - 1] + u[pa + 1]) + (u[pa - P] + u[pa + P])) + (u[pa - P2] + u[pa + P2]);
  const T sb = ((u[pb - 1] + u[pb + 1]) + (u[pb - P] + u[pb + P])) + (u[pb - P2] + u[pb + P2]);
  const T ra = rhs[ca], rb = rhs[cb];
  if (a.v) u[pa] = (sa - h2 * ra) * (col ? a.inv1 : a.inv0);
  if (b.v) u[pb] = (sb - h2 * rb) * (col ? b.inv1 : b.inv0);
}

// nu red-black sweeps in place, red ((x + y + z) even) first; u padded
template <class T>
__device__ void blk_gs(T* u, const T* rhs, int n, int nu) {
  if (nu <= 0) return;
  const double h = 1.0 / (double)n;
  const T h2 = (T)(h * h);
  const int P = n + 2, P2 = P * P, half = n * n * (n >> 1);
  const int NT = blockDim.x, t = threadIdx.x;
  const GsCell<T> a = gs_cell<T>(t, n, half), b = gs_cell<T>(t + NT, n, half);
  for (int it = 0; it < nu; ++it)
    for (int col = 0; col < 2; ++col) {
      if (a.v) gs_pair(u, rhs, P, P2, h2, col, a, b);
      for (int base = 2 * NT; base < half; base += 2 * NT) {  // levels above 4 NT cells
        const GsCell<T> e = gs_cell<T>(base + t, n, half), f = gs_cell<T>(base + t + NT, n, half);
        if (e.v) gs_pair(u, rhs, P, P2, h2, col, e, f);
      }
      __syncthreads();
    }
}

// uc = R u, rc = R (rhs - L u) on every coarse cell; then t = uc and
// rc = rc + L_H uc (FAS right-hand side, Eq. 4).  u, uc padded.
template <class T>
__device__ void blk_descend(const T* u, const T* rhs, int n, T* uc, T* rc, T* tc) {
  const int nc = n / 2, cc = nc * nc * nc;
  const int P = n + 2, P2 = P * P;
  const double s2 = (double)n * (double)n;
  Walk3 w(threadIdx.x, blockDim.x, nc, nc, cc);  // (I, J, K) of coarse cell c
  for (int c = threadIdx.x; c < cc; c += blockDim.x, w.next()) {
    const int K = w.k, J = w.j, I = w.i;
    double su = 0.0, sr = 0.0;
#pragma unroll
    for (int ch = 0; ch < 8; ++ch) {
      const int i = 2 * I + (ch & 1), j = 2 * J + ((ch >> 1) & 1), k = 2 * K + (ch >> 2);
      const int p = pidx(n, i, j, k);
      const double v = (double)u[p];
      const double s = (((double)u[p - 1] + (double)u[p + 1]) +
                         ((double)u[p - P] + (double)u[p + P])) +
                       ((double)u[p - P2] + (double)u[p + P2]);
      const int nb = (i == 0) + (i == n - 1) + (j == 0) + (j == n - 1) + (k == 0) + (k == n - 1);
      su += v;
      sr += (double)rhs[(k * n + j) * n + i] - (s - (double)(6 + nb) * v) * s2;
    }
    uc[pidx(nc, I, J, K)] = (T)(su / 8.0);
    rc[c] = (T)(sr / 8.0);
  }
  __syncthreads();
  const int Pc = nc + 2, Pc2 = Pc * Pc;
  const double sc2 = (double)nc * (double)nc;
  Walk3 w2(threadIdx.x, blockDim.x, nc, nc, cc);
  for (int c = threadIdx.x; c < cc; c += blockDim.x, w2.next()) {
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

// u += P(w - t): the increment of each coarse cell goes to its 8 children;
// u and w padded, t plain
template <class T>
__device__ void blk_correct(T* u, int n, const T* w, const T* t) {
  const int nc = n / 2, cc = nc * nc * nc;
  const int P = n + 2, P2 = P * P;
  Walk3 wk(threadIdx.x, blockDim.x, nc, nc, cc);
  for (int c = threadIdx.x; c < cc; c += blockDim.x, wk.next()) {
    const int K = wk.k, J = wk.j, I = wk.i;
    const T d = w[pidx(nc, I, J, K)] - t[c];
    const int p = pidx(n, 2 * I, 2 * J, 2 * K);
    T v[8];
#pragma unroll
    for (int ch = 0; ch < 8; ++ch) v[ch] = u[p + (ch >> 2) * P2 + ((ch >> 1) & 1) * P + (ch & 1)];
#pragma unroll
    for (int ch = 0; ch < 8; ++ch)
      u[p + (ch >> 2) * P2 + ((ch >> 1) & 1) * P + (ch & 1)] = (T)(v[ch] + d);
  }
  __syncthreads();
}

// FMG interpolation Pi (trilinear, odd reflection at the boundary) of the
// padded coarse c onto the padded fine u
template <class T>
__device__ void blk_interp(T* u, int n, const T* c) {
  const int cnt = n * n * n, nc = n / 2;
  Walk3 w(threadIdx.x, blockDim.x, n, n, cnt);
  for (int i = threadIdx.x; i < cnt; i += blockDim.x, w.next()) {
    const int x = w.i, y = w.j, z = w.k;
    const int f[3] = {x, y, z};
    int p[3], r[3];
    for (int d = 0; d < 3; ++d) {
      p[d] = f[d] >> 1;
      r[d] = (f[d] & 1) ? p[d] + 1 : p[d] - 1;
    }
    T s = 0;
    for (int cz = 0; cz < 2; ++cz)
      for (int cy = 0; cy < 2; ++cy)
        for (int cx = 0; cx < 2; ++cx) {
          int id3[3] = {cx ? r[0] : p[0], cy ? r[1] : p[1], cz ? r[2] : p[2]};
          T w = (T)((cx ? 0.25 : 0.75) * (cy ? 0.25 : 0.75) * (cz ? 0.25 : 0.75));
          T sign = 1;
          for (int d = 0; d < 3; ++d) {
            if (id3[d] < 0) { id3[d] = -1 - id3[d]; sign = -sign; }
            else if (id3[d] >= nc) { id3[d] = 2 * nc - 1 - id3[d]; sign = -sign; }
          }
          s += w * sign * c[pidx(nc, id3[0], id3[1], id3[2])];
        }
    u[pidx(n, x, y, z)] = s;
  }
  __syncthreads();
}

// exact coarsest solve u0 = A^-1 rhs0 (rhs0 plain, u0 padded)
template <class T>
__device__ void blk_coarse_solve(T* u0, const T* rhs0, int n0, const double* Ainv, int mm) {
  for (int r = threadIdx.x; r < mm; r += blockDim.x) {
    double s = 0.0;
    for (int c = 0; c < mm; ++c) s += Ainv[r * mm + c] * (double)rhs0[c];
    const int z = r / (n0 * n0), y = (r - z * n0 * n0) / n0, x = r - (z * n0 + y) * n0;
    u0[pidx(n0, x, y, z)] = (T)s;
  }
  __syncthreads();
}

// LDS elements k_coarse needs for levels 0..top with the given edges
__host__ __device__ inline int coarse_lds_elems(const int* n, int top, int mode) {
  int e = 0;
  for (int l = 0; l <= top; ++l) {
    const int c = n[l] * n[l] * n[l];
    e += coarse_padded(n[l]);  // u
    if (l < top) e += 2 * c;   // t, r
    if (mode == 0) e += c;     // f
  }
  if (mode == 1) e += n[top] * n[top] * n[top];  // rhs of the top level
  return e;
}

// Level data live in one LDS array; per-level offsets are kept in LDS too,
// so every access is an LDS instruction (no pointer tables in scratch).
struct CoarseOffsets {
  int u[kCoarseMaxLevels], t[kCoarseMaxLevels], r[kCoarseMaxLevels], f[kCoarseMaxLevels];
  int rt, uend;
};

// FAS V-cycle from level top with right-hand side sm + rto, down to the
// exact coarsest solve and back up
template <class T>
__device__ void blk_vcycle(T* sm, const CoarseOffsets& o, const CoarseArgs<T>& g, int top,
                           int rto) {
  for (int l = top; l >= 1; --l) {
    T* rhs = sm + ((l == top) ? rto : o.r[l]);
    blk_gs(sm + o.u[l], rhs, g.n[l], g.nu1);
    blk_descend(sm + o.u[l], rhs, g.n[l], sm + o.u[l - 1], sm + o.r[l - 1], sm + o.t[l - 1]);
  }
  blk_coarse_solve(sm + o.u[0], sm + (top == 0 ? rto : o.r[0]), g.n[0], g.Ainv, g.mm);
  for (int l = 1; l <= top; ++l) {
    T* rhs = sm + ((l == top) ? rto : o.r[l]);
    blk_correct(sm + o.u[l], g.n[l], sm + o.u[l - 1], sm + o.t[l - 1]);
    blk_gs(sm + o.u[l], rhs, g.n[l], g.nu2);
  }
}

// FAS right-hand side of the top level in LDS: r += L u (Eq. 2, in FP64) on
// every cell, and t = u to global memory; u padded, r plain
template <class T>
__device__ void blk_fas_rhs(const T* u, T* r, T* t, int n) {
  const int cnt = n * n * n, P = n + 2, P2 = P * P;
  const double s2 = (double)n * (double)n;
  Walk3 w(threadIdx.x, blockDim.x, n, n, cnt);
  for (int c = threadIdx.x; c < cnt; c += blockDim.x, w.next()) {
    const int x = w.i, y = w.j, z = w.k;
    const int p = pidx(n, x, y, z);
    const double v = (double)u[p];
    const double s = (((double)u[p - 1] + (double)u[p + 1]) + ((double)u[p - P] + (double)u[p + P])) +
                     ((double)u[p - P2] + (double)u[p + P2]);
    const int nb = (x == 0) + (x == n - 1) + (y == 0) + (y == n - 1) + (z == 0) + (z == n - 1);
    t[c] = u[p];
    r[c] = (T)((double)r[c] + (s - (double)(6 + nb) * v) * s2);
  }
  __syncthreads();
}

// copy an n^3 level between global memory (plain) and LDS (padded or plain);
// up to four loads per thread are in flight before the stores
template <class T, bool IN, bool PAD>
__device__ void blk_copy(T* lds, T* glob, int n) {
  const int cnt = n * n * n, NT = blockDim.x;
  Walk3 w(threadIdx.x, NT, n, n, cnt);
  for (int base = 0; base < cnt; base += 4 * NT) {
    T v[4];
    int li[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int i = base + threadIdx.x + k * NT;
      const bool in = i < cnt;
      li[k] = !in ? 0 : PAD ? pidx(n, w.i, w.j, w.k) : i;
      w.next();
      v[k] = in ? (IN ? glob[i] : lds[li[k]]) : (T)0;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int i = base + threadIdx.x + k * NT;
      if (i < cnt) {
        if (IN) lds[li[k]] = v[k];
        else glob[i] = v[k];
      }
    }
  }
}

// the right-hand side (plain) and u (padded) of an n^3 level from global
// memory into LDS, all loads of both issued before the stores
template <class T>
__device__ void blk_load_rhs_u(T* lr, const T* gr, T* lu, const T* gu, int n) {
  const int cnt = n * n * n, NT = blockDim.x;
  Walk3 w(threadIdx.x, NT, n, n, cnt);
  for (int base = 0; base < cnt; base += 4 * NT) {
    T vr[4], vu[4];
    int li[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int i = base + threadIdx.x + k * NT;
      const bool in = i < cnt;
      li[k] = in ? pidx(n, w.i, w.j, w.k) : 0;
      w.next();
      vr[k] = in ? gr[i] : (T)0;
      vu[k] = in ? gu[i] : (T)0;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int i = base + threadIdx.x + k * NT;
      if (i < cnt) {
        lr[i] = vr[k];
        lu[li[k]] = vu[k];
      }
    }
  }
}

// f of level l - 1 = R f of level l (mean of the 8 children, summed in FP64
// in the order of the global restriction kernel); both plain, in LDS
template <class T>
__device__ void blk_restrict_f(const T* f, int n, T* fc) {
  const int nc = n / 2, cnt = nc * nc * nc;
  Walk3 w(threadIdx.x, blockDim.x, nc, nc, cnt);
  for (int c = threadIdx.x; c < cnt; c += blockDim.x, w.next()) {
    double s = 0.0;
    for (int k = 0; k < 2; ++k)
      for (int j = 0; j < 2; ++j)
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
  Walk3 w(threadIdx.x, blockDim.x, n, n, cnt);
  for (int i = threadIdx.x; i < cnt; i += blockDim.x, w.next())
    out[i] = (double)lds[pidx(n, w.i, w.j, w.k)];
}

template <class T>
__global__ void __launch_bounds__(kCoarseThreads) k_coarse(CoarseArgs<T> g) {
  extern __shared__ unsigned char smem_raw[];
  T* sm = reinterpret_cast<T*>(smem_raw);
  __shared__ CoarseOffsets o;
  if (threadIdx.x == 0) {
    int off = 0;
    for (int l = 0; l <= g.top; ++l) {
      o.u[l] = off;
      off += coarse_padded(g.n[l]);
    }
    o.uend = off;
    for (int l = 0; l <= g.top; ++l) {
      const int c = g.n[l] * g.n[l] * g.n[l];
      o.t[l] = o.r[l] = o.f[l] = 0;
      if (l < g.top) {
        o.t[l] = off;
        off += c;
        o.r[l] = off;
        off += c;
      }
    }
    if (g.mode == 0) {
      for (int l = 0; l <= g.top; ++l) {
        o.f[l] = off;
        off += g.n[l] * g.n[l] * g.n[l];
      }
    }
    o.rt = off;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < o.uend; i += blockDim.x) sm[i] = (T)0;  // halos
  __syncthreads();
  if (g.mode == 0) {  // f of the top level; the coarser ones are restricted here
    blk_copy<T, true, false>(sm + o.f[g.top], const_cast<T*>(g.f[g.top]), g.n[g.top]);
  } else {
    blk_load_rhs_u(sm + o.rt, g.rt, sm + o.u[g.top], g.u[g.top], g.n[g.top]);
  }
  __syncthreads();
  if (g.mode == 0)
    for (int l = g.top; l >= 1; --l) blk_restrict_f(sm + o.f[l], g.n[l], sm + o.f[l - 1]);
  if (g.mode == 1) {
    if (g.fas) blk_fas_rhs(sm + o.u[g.top], sm + o.rt, g.t[g.top], g.n[g.top]);
    blk_vcycle(sm, o, g, g.top, o.rt);
  } else {
    blk_coarse_solve(sm + o.u[0], sm + o.f[0], g.n[0], g.Ainv, g.mm);
    if (g.ck[0]) blk_checkpoint(sm + o.u[0], g.ck[0], g.n[0]);
    for (int l = 1; l <= g.top; ++l) {
      blk_interp(sm + o.u[l], g.n[l], sm + o.u[l - 1]);
      blk_gs(sm + o.u[l], sm + o.f[l], g.n[l], g.alpha);
      blk_vcycle(sm, o, g, l, o.f[l]);
      if (g.ck[l]) blk_checkpoint(sm + o.u[l], g.ck[l], g.n[l]);
    }
  }
  blk_copy<T, false, true>(sm + o.u[g.top], g.u[g.top], g.n[g.top]);
}

}  // namespace fmg
