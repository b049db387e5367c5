// kernels_coarse.hpp -- the coarse global levels in one persistent workgroup.
//
// Levels whose grids are small (up to 16^3 cells) are latency bound: a kernel
// launch per operator costs more than the work.  k_coarse runs every
// operator of these levels inside one workgroup, with a block barrier between
// phases, on copies of the levels held in LDS: it loads what the cycle reads
// (the top level's u and right-hand side, or the FMG right-hand sides), works
// in LDS and writes back the top level's u, the only result used outside.
// It performs either
//   mode 0: FMG stages 0..top (Fig. 2 of the paper): u_0 = L_0^-1 f_0, then
//           per level Pi, S^alpha and one FAS V-cycle with rhs f_l, or
//   mode 1: one FAS V-cycle (Fig. 1) on level top with right-hand side rt.
// Every phase applies exactly the per-cell arithmetic of the single-cell
// kernels; updates of one colour are independent, so the in-place half-sweep
// is an exact Gauss-Seidel half-sweep.
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
  const T* rt;  // mode 1: rhs of level top
  int nu1, nu2, alpha;
};

// 1 / (6 + nb) for nb = 0..6 boundary faces (constants, no division)
template <class T>
__device__ inline T inv_diag(int nb) {
  return nb == 0 ? (T)(1.0 / 6.0) : nb == 1 ? (T)(1.0 / 7.0) : nb == 2 ? (T)(1.0 / 8.0)
       : nb == 3 ? (T)(1.0 / 9.0) : nb == 4 ? (T)(1.0 / 10.0) : nb == 5 ? (T)(1.0 / 11.0)
       : (T)(1.0 / 12.0);
}

// Cells of an n^3 level owned by this thread: column (x, y) and planes
// z0, z0 + zs, ... (zs threads share a column); returns false when idle.
__device__ inline bool blk_column(int n, int& x, int& y, int& z0, int& zs) {
  const int n2 = n * n;
  zs = (int)blockDim.x / n2;
  if (zs < 1) zs = 1;
  const int t = threadIdx.x;
  if (t >= n2 * zs) return false;
  const int c = t % n2;
  z0 = t / n2;
  y = c / n;
  x = c - y * n;
  return true;
}

// nu red-black sweeps in place (n <= 32 so every column has an owner)
template <class T>
__device__ void blk_gs(T* u, const T* rhs, int n, int nu) {
  const double h = 1.0 / (double)n;
  const T h2 = (T)(h * h);
  int x = 0, y = 0, z0 = 0, zs = 1;
  const bool on = blk_column(n, x, y, z0, zs);
  const int n2 = n * n;
  const int bxy = (x == 0) + (x == n - 1) + (y == 0) + (y == n - 1);
  for (int it = 0; it < nu; ++it)
    for (int col = 0; col < 2; ++col) {
      if (on) {
        for (int z = z0; z < n; z += zs) {
          if (((x + y + z) & 1) != col) continue;
          const int c = (z * n + y) * n + x;
          T s = 0;
          if (x > 0) s += u[c - 1];
          if (x < n - 1) s += u[c + 1];
          if (y > 0) s += u[c - n];
          if (y < n - 1) s += u[c + n];
          if (z > 0) s += u[c - n2];
          if (z < n - 1) s += u[c + n2];
          const int nb = bxy + (z == 0) + (z == n - 1);
          u[c] = (s - h2 * rhs[c]) * inv_diag<T>(nb);
        }
      }
      __syncthreads();
    }
}

// uc = R u, rc = R (rhs - L u) on every coarse cell; then t = uc and
// rc = rc + L_H uc (FAS right-hand side, Eq. 4)
template <class T>
__device__ void blk_descend(const T* u, const T* rhs, int n, T* uc, T* rc, T* tc) {
  const Geo G = global_geo(n);
  const Box B = seg_box(G, 0);
  const int nc = n / 2, nc2 = nc * nc;
  const int cc = nc * nc2;
  for (int c = threadIdx.x; c < cc; c += blockDim.x) {
    int K = c / nc2, J = (c - K * nc2) / nc, I = c - K * nc2 - J * nc;
    double su = 0.0, sr = 0.0;
    for (int cz = 0; cz < 2; ++cz)
      for (int cy = 0; cy < 2; ++cy)
        for (int cx = 0; cx < 2; ++cx) {
          int i = 2 * I + cx, j = 2 * J + cy, k = 2 * K + cz;
          int id = (k * n + j) * n + i;
          su += (double)u[id];
          sr += (double)rhs[id] - apply_L<T, double>(u, G, B, i, j, k);
        }
    uc[c] = (T)(su / 8.0);
    rc[c] = (T)(sr / 8.0);
  }
  __syncthreads();
  const Geo Gc = global_geo(nc);
  const Box Bc = seg_box(Gc, 0);
  for (int c = threadIdx.x; c < cc; c += blockDim.x) {
    int K = c / nc2, J = (c - K * nc2) / nc, I = c - K * nc2 - J * nc;
    tc[c] = uc[c];
    rc[c] = (T)((double)rc[c] + apply_L<T, double>(uc, Gc, Bc, I, J, K));
  }
  __syncthreads();
}

// u += P(w - t): the increment is formed per fine cell from the coarse pair
template <class T>
__device__ void blk_correct(T* u, int n, const T* w, const T* t) {
  const int nc = n / 2;
  int x = 0, y = 0, z0 = 0, zs = 1;
  if (blk_column(n, x, y, z0, zs)) {
    for (int z = z0; z < n; z += zs) {
      const int pc = ((z >> 1) * nc + (y >> 1)) * nc + (x >> 1);
      const int c = (z * n + y) * n + x;
      u[c] = (T)(u[c] + (w[pc] - t[pc]));
    }
  }
  __syncthreads();
}

template <class T>
__device__ void blk_interp(T* u, int n, const T* c) {
  const Geo G = global_geo(n), Gc = global_geo(n / 2);
  const Box Bc = seg_box(Gc, 0);
  const int n2 = n * n, cnt = n * n2;
  for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
    int z = i / n2, y = (i - z * n2) / n, x = i - z * n2 - y * n;
    int f[3] = {x, y, z};
    int nc = n / 2, p[3], r[3];
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
          s += w * sign * c[at(Gc, Bc, id3[0], id3[1], id3[2])];
        }
    u[i] = s;
  }
  (void)G;
  __syncthreads();
}

template <class T>
__device__ void blk_coarse_solve(T* u0, const T* rhs0, const double* Ainv, int mm) {
  for (int r = threadIdx.x; r < mm; r += blockDim.x) {
    double s = 0.0;
    for (int c = 0; c < mm; ++c) s += Ainv[r * mm + c] * (double)rhs0[c];
    u0[r] = (T)s;
  }
  __syncthreads();
}

// LDS elements k_coarse needs for levels 0..top with the given edges
__host__ __device__ inline int coarse_lds_elems(const int* n, int top, int mode) {
  int e = 0;
  for (int l = 0; l <= top; ++l) {
    int c = n[l] * n[l] * n[l];
    e += c;                          // u
    if (l < top) e += 2 * c;         // t, r
    if (mode == 0) e += c;           // f
  }
  if (mode == 1) e += n[top] * n[top] * n[top];  // rhs of the top level
  return e;
}

// Level data live in one LDS array; per-level offsets are kept in LDS too,
// so every access is an LDS instruction (no pointer tables in scratch).
struct CoarseOffsets {
  int u[kCoarseMaxLevels], t[kCoarseMaxLevels], r[kCoarseMaxLevels], f[kCoarseMaxLevels];
  int rt;
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
  blk_coarse_solve(sm + o.u[0], sm + (top == 0 ? rto : o.r[0]), g.Ainv, g.mm);
  for (int l = 1; l <= top; ++l) {
    T* rhs = sm + ((l == top) ? rto : o.r[l]);
    blk_correct(sm + o.u[l], g.n[l], sm + o.u[l - 1], sm + o.t[l - 1]);
    blk_gs(sm + o.u[l], rhs, g.n[l], g.nu2);
  }
}

template <class T>
__global__ void __launch_bounds__(kCoarseThreads) k_coarse(CoarseArgs<T> g) {
  extern __shared__ unsigned char smem_raw[];
  T* sm = reinterpret_cast<T*>(smem_raw);
  __shared__ CoarseOffsets o;
  if (threadIdx.x == 0) {
    int off = 0;
    for (int l = 0; l <= g.top; ++l) {
      int c = g.n[l] * g.n[l] * g.n[l];
      o.u[l] = off;
      off += c;
      o.t[l] = o.r[l] = 0;
      if (l < g.top) {
        o.t[l] = off;
        off += c;
        o.r[l] = off;
        off += c;
      }
      o.f[l] = 0;
      if (g.mode == 0) {
        o.f[l] = off;
        off += c;
      }
    }
    o.rt = off;
  }
  __syncthreads();
  const int ct = g.n[g.top] * g.n[g.top] * g.n[g.top];
  if (g.mode == 0) {
    for (int l = 0; l <= g.top; ++l) {
      const int c = g.n[l] * g.n[l] * g.n[l];
      const T* src = g.f[l];
      T* dst = sm + o.f[l];
      for (int i = threadIdx.x; i < c; i += blockDim.x) dst[i] = src[i];
    }
  } else {
    const T* rt = g.rt;
    const T* ut = g.u[g.top];
    T* drt = sm + o.rt;
    T* dut = sm + o.u[g.top];
    for (int i = threadIdx.x; i < ct; i += blockDim.x) {
      drt[i] = rt[i];
      dut[i] = ut[i];
    }
  }
  __syncthreads();
  if (g.mode == 1) {
    blk_vcycle(sm, o, g, g.top, o.rt);
  } else {
    blk_coarse_solve(sm + o.u[0], sm + o.f[0], g.Ainv, g.mm);
    for (int l = 1; l <= g.top; ++l) {
      blk_interp(sm + o.u[l], g.n[l], sm + o.u[l - 1]);
      blk_gs(sm + o.u[l], sm + o.f[l], g.n[l], g.alpha);
      blk_vcycle(sm, o, g, l, o.f[l]);
    }
  }
  T* ut = g.u[g.top];
  const T* su = sm + o.u[g.top];
  for (int i = threadIdx.x; i < ct; i += blockDim.x) ut[i] = su[i];
}

}  // namespace fmg
