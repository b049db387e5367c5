// kernels_simple.hpp -- one-thread-per-cell kernels for every operator of the
// solve.  They run every level that the fused LDS kernels do not take, and
// the single-operator entry points.
//
// Template parameters: T is the storage type (double, or float for the FP32
// multigrid of the mixed-precision solve); A is the arithmetic type of an
// operation (the residual and the restriction always accumulate in double).
//
// Operators (paper, Sec. 2 and 3):
//   L_h u   = h^-2 (sum of 6 neighbours - 6 u_c), a neighbour outside the
//             domain being the ghost -u_c (u = 0 on the face);
//   GS      = exact solve of row c: u_c = (sum of in-domain neighbours
//             - h^2 rhs_c) / (6 + b_c), b_c = faces of c on the boundary;
//   R       = mean of the 8 children;  P = parent's value;
//   Pi      = trilinear, 1D weights 3/4 (parent) and 1/4 (next coarse cell
//             on the child's side), odd reflection outside the domain.
#pragma once
#include "grid.hpp"

namespace fmg {

// sum of the in-domain neighbours of (i,j,k) and the number of boundary faces
template <class T, class A>
__device__ inline A nb_sum(const T* __restrict__ u, const Geo& G, const Box& B, int i, int j,
                           int k, int& nb) {
  A s = 0;
  nb = 0;
  const int n = G.n;
  if (i > 0) s += (A)u[at(G, B, i - 1, j, k)]; else ++nb;
  if (i < n - 1) s += (A)u[at(G, B, i + 1, j, k)]; else ++nb;
  if (j > 0) s += (A)u[at(G, B, i, j - 1, k)]; else ++nb;
  if (j < n - 1) s += (A)u[at(G, B, i, j + 1, k)]; else ++nb;
  if (k > 0) s += (A)u[at(G, B, i, j, k - 1)]; else ++nb;
  if (k < n - 1) s += (A)u[at(G, B, i, j, k + 1)]; else ++nb;
  return s;
}

// (L_h u) at an in-domain cell
template <class T, class A>
__device__ inline A apply_L(const T* __restrict__ u, const Geo& G, const Box& B, int i, int j,
                            int k) {
  int nb;
  A s = nb_sum<T, A>(u, G, B, i, j, k, nb);
  A uc = (A)u[at(G, B, i, j, k)];
  return (s - (A)(6 + nb) * uc) * ((A)G.n * (A)G.n);
}

// cell of a box extent from a linear thread index; false when past the end
__device__ inline bool cell_of(long long t, int ex, int ey, int ez, int& x, int& y, int& z) {
  long long cnt = (long long)ex * ey * ez;
  if (t >= cnt) return false;
  x = (int)(t % ex);
  long long r = t / ex;
  y = (int)(r % ey);
  z = (int)(r / ey);
  return true;
}

// ---------------------------------------------------------------------------
// red-black Gauss-Seidel half-sweep of colour col over C of every segment.
// rhs may live on a global view (gr) while u is segmented (gu).
template <class T, class A>
__global__ void k_gs_half(T* __restrict__ u, Geo gu, const T* __restrict__ rhs, Geo gr, int col,
                          A h2, int ce) {
  int q = blockIdx.y;
  Box B = seg_box(gu, q), Br = seg_box(gr, q);
  int x, y, z;
  if (!cell_of((long long)blockIdx.x * blockDim.x + threadIdx.x, ce, ce, ce, x, y, z)) return;
  int i = B.a[0] + x, j = B.a[1] + y, k = B.a[2] + z;
  if (i >= B.b[0] || j >= B.b[1] || k >= B.b[2]) return;
  if (((i + j + k) & 1) != col) return;
  int nb;
  A s = nb_sum<T, A>(u, gu, B, i, j, k, nb);
  A r = (A)rhs[at(gr, Br, i, j, k)];
  u[at(gu, B, i, j, k)] = (T)((s - h2 * r) / (A)(6 + nb));
}

// out = L_h u on a global level (single-operator entry point)
template <class T>
__global__ void k_apply(const T* __restrict__ u, Geo G, T* __restrict__ out) {
  Box B = seg_box(G, 0);
  int x, y, z;
  if (!cell_of((long long)blockIdx.x * blockDim.x + threadIdx.x, G.n, G.n, G.n, x, y, z)) return;
  out[at(G, B, x, y, z)] = (T)apply_L<T, double>(u, G, B, x, y, z);
}

// ---------------------------------------------------------------------------
// Residual and restriction.  For every coarse cell of the target region:
//   uc = R u (solution restriction, Fig. 1 and Fig. 6) and
//   rc = R (rhs - L_h u) (residual restriction),
// where the children's residuals are formed on the fine level.
// mode 0: target = F = C_fine / 2 of the same segment (global V-cycle: the
//         whole coarse level);
// mode 1: target = the genuine cells of segment q on the transition level
//         (owner computes; coarse views are global).
template <class T>
__global__ void k_resid_restrict(const T* __restrict__ u, Geo gu, const T* __restrict__ rhs,
                                 Geo gr, T* __restrict__ uc, T* __restrict__ rc, Geo gc,
                                 int mode, int ce) {
  int q = blockIdx.y;
  Box B = seg_box(gu, q), Br = seg_box(gr, q), Bc = seg_box(gc, q);
  int lo[3], hi[3];
  if (mode == 0) {
    for (int d = 0; d < 3; ++d) { lo[d] = B.a[d] / 2; hi[d] = B.b[d] / 2; }
  } else {
    int S = gu.S, e = gc.n / S;
    int p[3] = {q % S, (q / S) % S, q / (S * S)};
    for (int d = 0; d < 3; ++d) { lo[d] = p[d] * e; hi[d] = (p[d] + 1) * e; }
  }
  int x, y, z;
  if (!cell_of((long long)blockIdx.x * blockDim.x + threadIdx.x, ce, ce, ce, x, y, z)) return;
  int I = lo[0] + x, J = lo[1] + y, K = lo[2] + z;
  if (I >= hi[0] || J >= hi[1] || K >= hi[2]) return;
  double su = 0.0, sr = 0.0;
  for (int c = 0; c < 2; ++c)
    for (int b = 0; b < 2; ++b)
      for (int a = 0; a < 2; ++a) {
        int i = 2 * I + a, j = 2 * J + b, k = 2 * K + c;
        su += (double)u[at(gu, B, i, j, k)];
        sr += (double)rhs[at(gr, Br, i, j, k)] - apply_L<T, double>(u, gu, B, i, j, k);
      }
  uc[at(gc, Bc, I, J, K)] = (T)(su / 8.0);
  rc[at(gc, Bc, I, J, K)] = (T)(sr / 8.0);
}

// Coarse right-hand side of the FAS cycle after the restriction:
//   t = u over the whole coarse box (compute region and ghosts);
//   rhs = rc + L_H u on F, rhs = L_H u on C \ F (Fig. 6; rc holds R res on F
//   on entry and rhs on exit).  whole_f: F covers the whole level (global
//   levels and the transition level).
template <class T>
__global__ void k_coarse_rhs(const T* __restrict__ uc, T* __restrict__ rc, T* __restrict__ tc,
                             Geo gc, Geo gf, int whole_f) {
  int q = blockIdx.y;
  Box Bc = seg_box(gc, q);
  int me = gc.m;
  int x, y, z;
  if (!cell_of((long long)blockIdx.x * blockDim.x + threadIdx.x, me, me, me, x, y, z)) return;
  int I = Bc.o[0] + x, J = Bc.o[1] + y, K = Bc.o[2] + z;
  long long id = at(gc, Bc, I, J, K);
  tc[id] = uc[id];
  if (I < Bc.a[0] || I >= Bc.b[0] || J < Bc.a[1] || J >= Bc.b[1] || K < Bc.a[2] || K >= Bc.b[2])
    return;
  bool inF = true;
  if (!whole_f) {
    Box Bf = seg_box(gf, q);
    inF = I >= Bf.a[0] / 2 && I < Bf.b[0] / 2 && J >= Bf.a[1] / 2 && J < Bf.b[1] / 2 &&
          K >= Bf.a[2] / 2 && K < Bf.b[2] / 2;
  }
  double Lu = apply_L<T, double>(uc, gc, Bc, I, J, K);
  double r = inF ? (double)rc[id] : 0.0;
  rc[id] = (T)(r + Lu);
}

// u += P(w - t) on C and the GSR ghosts (every stored cell inside the domain)
template <class T>
__global__ void k_correct(T* __restrict__ u, Geo gu, const T* __restrict__ w,
                          const T* __restrict__ t, Geo gc) {
  int q = blockIdx.y;
  Box B = seg_box(gu, q), Bc = seg_box(gc, q);
  int me = gu.m;
  int x, y, z;
  if (!cell_of((long long)blockIdx.x * blockDim.x + threadIdx.x, me, me, me, x, y, z)) return;
  int i = B.o[0] + x, j = B.o[1] + y, k = B.o[2] + z;
  if (!in_dom(gu.n, i, j, k)) return;
  long long pc = at(gc, Bc, i >> 1, j >> 1, k >> 1);
  long long id = at(gu, B, i, j, k);
  u[id] = (T)(u[id] + (w[pc] - t[pc]));
}

// FMG interpolation onto C and the GSR ghosts
template <class T>
__global__ void k_interp(T* __restrict__ u, Geo gu, const T* __restrict__ c, Geo gc) {
  int q = blockIdx.y;
  Box B = seg_box(gu, q), Bc = seg_box(gc, q);
  int me = gu.m;
  int x, y, z;
  if (!cell_of((long long)blockIdx.x * blockDim.x + threadIdx.x, me, me, me, x, y, z)) return;
  int f[3] = {B.o[0] + x, B.o[1] + y, B.o[2] + z};
  if (!in_dom(gu.n, f[0], f[1], f[2])) return;
  int nc = gc.n;
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
        s += w * sign * c[at(gc, Bc, id3[0], id3[1], id3[2])];
      }
  u[at(gu, B, f[0], f[1], f[2])] = s;
}

// global level: coarse = mean of children (right-hand-side hierarchy)
template <class Tf, class Tc>
__global__ void k_restrict_global(const Tf* __restrict__ fine, int n, Tc* __restrict__ coarse) {
  int nc = n / 2;
  int X, Y, Z;
  if (!cell_of((long long)blockIdx.x * blockDim.x + threadIdx.x, nc, nc, nc, X, Y, Z)) return;
  double s = 0.0;
  for (int c = 0; c < 2; ++c)
    for (int b = 0; b < 2; ++b)
      for (int a = 0; a < 2; ++a)
        s += (double)fine[((long long)(2 * Z + c) * n + (2 * Y + b)) * n + (2 * X + a)];
  coarse[((long long)Z * nc + Y) * nc + X] = (Tc)(s / 8.0);
}

// the right-hand-side hierarchy several levels at once: a workgroup reads a
// (2 << depth)^3 block of the fine level once and writes the matching blocks
// of the next depth coarser levels (c0 the next, c3 the fourth), each a mean
// of 8 children summed in the order of k_restrict_global, the intermediate
// levels kept in LDS.  depth 1..4; n divisible by 2 << depth.
template <class T>
__global__ void __launch_bounds__(1024) k_restrict_chain(const T* __restrict__ fine, int n, int depth,
                                                         T* c0, T* c1, T* c2, T* c3) {
  __shared__ T la[16 * 16 * 16], lb[8 * 8 * 8];
  const int E = 2 << depth, nb = n / E;
  const int bx = blockIdx.x % nb, by = (blockIdx.x / nb) % nb, bz = blockIdx.x / (nb * nb);
  int e = E >> 1, nl = n >> 1;  // block and level edge of the level being written
  for (int c = threadIdx.x; c < e * e * e; c += blockDim.x) {
    const int X = c % e, Y = (c / e) % e, Z = c / (e * e);
    const long long gx = (long long)bx * E + 2 * X, gy = (long long)by * E + 2 * Y,
                    gz = (long long)bz * E + 2 * Z;
    double s = 0.0;
    for (int k = 0; k < 2; ++k)
      for (int j = 0; j < 2; ++j)
        for (int i = 0; i < 2; ++i) s += (double)fine[((gz + k) * n + (gy + j)) * n + (gx + i)];
    const T v = (T)(s / 8.0);
    c0[((long long)(bz * e + Z) * nl + (by * e + Y)) * nl + (bx * e + X)] = v;
    la[c] = v;
  }
  __syncthreads();
  T* src = la;
  T* dst = lb;
  for (int d = 1; d < depth; ++d) {
    const int ec = e >> 1, ncl = nl >> 1;
    T* out = d == 1 ? c1 : d == 2 ? c2 : c3;
    for (int c = threadIdx.x; c < ec * ec * ec; c += blockDim.x) {
      const int X = c % ec, Y = (c / ec) % ec, Z = c / (ec * ec);
      double s = 0.0;
      for (int k = 0; k < 2; ++k)
        for (int j = 0; j < 2; ++j)
          for (int i = 0; i < 2; ++i) s += (double)src[((2 * Z + k) * e + (2 * Y + j)) * e + (2 * X + i)];
      const T v = (T)(s / 8.0);
      out[((long long)(bz * ec + Z) * ncl + (by * ec + Y)) * ncl + (bx * ec + X)] = v;
      dst[c] = v;
    }
    __syncthreads();
    T* tmp = src;
    src = dst;
    dst = tmp;
    e = ec;
    nl = ncl;
  }
}

// coarsest level: u = A^-1 rhs with the FP64 inverse precomputed on the host
template <class T>
__global__ void k_coarse_solve(T* __restrict__ u, const T* __restrict__ rhs,
                               const double* __restrict__ Ainv, int mm) {
  for (int r = threadIdx.x; r < mm; r += blockDim.x) {
    double s = 0.0;
    for (int c = 0; c < mm; ++c) s += Ainv[(long long)r * mm + c] * (double)rhs[c];
    u[r] = (T)s;
  }
}

// genuine cells of every finest-level segment into the caller's N^3 array
template <class T>
__global__ void k_gather(double* __restrict__ out, const T* __restrict__ u, Geo gu, int acc) {
  int q = blockIdx.y;
  Box B = seg_box(gu, q);
  int S = gu.S, g = gu.g;
  int p[3] = {q % S, (q / S) % S, q / (S * S)};
  int x, y, z;
  if (!cell_of((long long)blockIdx.x * blockDim.x + threadIdx.x, g, g, g, x, y, z)) return;
  int i = p[0] * g + x, j = p[1] * g + y, k = p[2] * g + z;
  long long o = ((long long)k * gu.n + j) * gu.n + i;
  double v = (double)u[at(gu, B, i, j, k)];
  out[o] = acc ? out[o] + v : v;
}

// ---------------------------------------------------------------------------
// outer loop of the mixed-precision solve (FP64 residual and update)

// r = (float)(f - L_h u), all in FP64; has_u == 0 means u = 0.  A tile of
// kResTX x kResTY columns marches a z chunk of zc planes: each thread keeps
// its column's planes z - 1, z and z + 1 in registers, and its x and y
// neighbours are the same plane's loads of adjacent lanes and rows, so they
// come from the cache.  Neighbours are summed in the order of nb_sum.
constexpr int kResTX = 64, kResTY = 4;
__global__ void __launch_bounds__(kResTX * kResTY)
    k_resid64_to32(const double* __restrict__ f, const double* __restrict__ u, int has_u, int n,
                   int zc, float* __restrict__ r) {
  const int x = blockIdx.x * kResTX + (int)(threadIdx.x % kResTX);
  const int y = blockIdx.y * kResTY + (int)(threadIdx.x / kResTX);
  const int z0 = blockIdx.z * zc, z1 = min(n, z0 + zc);
  if (x >= n || y >= n) return;  // (no barrier follows)
  const long long nn = (long long)n * n, col = (long long)y * n + x;
  if (!has_u) {
    for (int z = z0; z < z1; ++z) r[z * nn + col] = (float)f[z * nn + col];
    return;
  }
  const double n2 = (double)n * (double)n;
  double um = z0 > 0 ? u[(z0 - 1) * nn + col] : 0.0;
  double uc = z0 < n ? u[z0 * nn + col] : 0.0;
  for (int z = z0; z < z1; ++z) {
    const long long id = z * nn + col;
    const double up = z + 1 < n ? u[id + nn] : 0.0;
    double s = 0.0;
    int nb = 0;
    if (x > 0) s += u[id - 1]; else ++nb;
    if (x < n - 1) s += u[id + 1]; else ++nb;
    if (y > 0) s += u[id - n]; else ++nb;
    if (y < n - 1) s += u[id + n]; else ++nb;
    if (z > 0) s += um; else ++nb;
    if (z < n - 1) s += up; else ++nb;
    const double v = f[id];
    r[id] = (float)(v - (s - (double)(6 + nb) * uc) * n2);
    um = uc;
    uc = up;
  }
}

// The FAS right-hand side of a global level whose F is the whole level
// (k_coarse_rhs there) as a z march: t = u and r = r + L u, one thread per
// column (x, y) over a chunk of zc planes, u's z neighbours carried in
// registers, the in-plane ones read through the cache.  Same arithmetic, in
// the same order, as k_coarse_rhs (nb_sum, apply_L).
template <class T>
__global__ void __launch_bounds__(kResTX * kResTY)
    k_coarse_rhs_z(const T* __restrict__ u, T* __restrict__ r, T* __restrict__ t, int n, int zc) {
  const int x = blockIdx.x * kResTX + (int)(threadIdx.x % kResTX);
  const int y = blockIdx.y * kResTY + (int)(threadIdx.x / kResTX);
  const int z0 = blockIdx.z * zc, z1 = min(n, z0 + zc);
  if (x >= n || y >= n) return;  // (no barrier follows)
  const long long nn = (long long)n * n, col = (long long)y * n + x;
  const double n2 = (double)n * (double)n;
  double um = z0 > 0 ? (double)u[(z0 - 1) * nn + col] : 0.0;
  T uv = u[z0 * nn + col];
  for (int z = z0; z < z1; ++z) {
    const long long id = z * nn + col;
    const T upv = z + 1 < n ? u[id + nn] : (T)0;
    const double uc = (double)uv, up = (double)upv;
    double s = 0.0;
    int nb = 0;
    if (x > 0) s += (double)u[id - 1]; else ++nb;
    if (x < n - 1) s += (double)u[id + 1]; else ++nb;
    if (y > 0) s += (double)u[id - n]; else ++nb;
    if (y < n - 1) s += (double)u[id + n]; else ++nb;
    if (z > 0) s += um; else ++nb;
    if (z < n - 1) s += up; else ++nb;
    t[id] = uv;
    r[id] = (T)((double)r[id] + (s - (double)(6 + nb) * uc) * n2);
    um = uc;
    uv = upv;
  }
}

// Residual and restriction of a global level onto the whole coarse global
// level (k_resid_restrict there, mode 0) as a z march: one thread per coarse
// column (X, Y) over a chunk of zc coarse planes.  The 2 x 2 fine columns
// under it carry u of fine planes 2Z - 1 .. 2Z + 2 in registers from one
// coarse plane to the next; in-plane neighbours outside the 2 x 2 block come
// through the cache.  Same arithmetic, in the same order, as
// k_resid_restrict (children z, y, x; nb_sum; apply_L).
template <class T>
__global__ void __launch_bounds__(kResTX * kResTY)
    k_resid_restrict_z(const T* __restrict__ u, const T* __restrict__ rhs, T* __restrict__ uc,
                       T* __restrict__ rc, int n, int zc) {
  const int nc = n / 2;
  const int X = blockIdx.x * kResTX + (int)(threadIdx.x % kResTX);
  const int Y = blockIdx.y * kResTY + (int)(threadIdx.x / kResTX);
  const int Z0 = blockIdx.z * zc, Z1 = min(nc, Z0 + zc);
  if (X >= nc || Y >= nc) return;  // (no barrier follows)
  const long long nn = (long long)n * n;
  const int x0 = 2 * X, y0 = 2 * Y;
  const long long c0 = (long long)y0 * n + x0;  // fine column (x0, y0)
  const double n2 = (double)n * (double)n;
  // w[p][b][a]: u at fine (x0 + a, y0 + b, 2Z - 1 + p), 0 outside the domain
  double w[4][2][2];
  auto load = [&](int k, double (&d)[2][2]) {
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int a = 0; a < 2; ++a)
        d[b][a] = (k >= 0 && k < n) ? (double)u[k * nn + c0 + b * n + a] : 0.0;
  };
  load(2 * Z0 - 1, w[0]);
  load(2 * Z0, w[1]);
  for (int Z = Z0; Z < Z1; ++Z) {
    load(2 * Z + 1, w[2]);
    load(2 * Z + 2, w[3]);
    double su = 0.0, sr = 0.0;
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int a = 0; a < 2; ++a) {
          const int i = x0 + a, j = y0 + b, k = 2 * Z + c;
          const long long id = k * nn + c0 + b * n + a;
          const double v = w[c + 1][b][a];
          su += v;
          double s = 0.0;
          int nb = 0;
          if (a == 1) s += w[c + 1][b][0]; else if (i > 0) s += (double)u[id - 1]; else ++nb;
          if (a == 0) s += w[c + 1][b][1]; else if (i < n - 1) s += (double)u[id + 1]; else ++nb;
          if (b == 1) s += w[c + 1][0][a]; else if (j > 0) s += (double)u[id - n]; else ++nb;
          if (b == 0) s += w[c + 1][1][a]; else if (j < n - 1) s += (double)u[id + n]; else ++nb;
          if (k > 0) s += w[c][b][a]; else ++nb;
          if (k < n - 1) s += w[c + 2][b][a]; else ++nb;
          sr += (double)rhs[id] - (s - (double)(6 + nb) * v) * n2;
        }
    const long long ic = ((long long)Z * nc + Y) * nc + X;
    uc[ic] = (T)(su / 8.0);
    rc[ic] = (T)(sr / 8.0);
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        w[0][b][a] = w[2][b][a];
        w[1][b][a] = w[3][b][a];
      }
  }
}

// u (+)= e
template <class T>
__global__ void k_update64(double* __restrict__ u, const T* __restrict__ e, long long cnt,
                           int acc) {
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= cnt) return;
  double v = (double)e[t];
  u[t] = acc ? u[t] + v : v;
}

}  // namespace fmg
