// kernels_cols.hpp -- the red-black smoother for small global levels, with
// every plane of a z chunk in registers.
//
// On levels of a few ten thousand cells a smoothing pass is a chain of memory
// round trips, not a stream: a z march that keeps a few planes in flight
// waits on one round trip every few steps.  k_smooth_cols takes one column
// per thread and holds the column's whole z chunk, halo planes included, in
// registers, so a pass costs one round of loads:
//
//  * a workgroup owns an xy tile of txw x tyw columns (halo H on each side)
//    and a chunk of ZC output planes with HZ halo planes below and above;
//  * every load of the chunk is issued before the first is used: u (or the
//    correction u + (w - t) of the parent, or the FMG interpolation of the
//    coarse level) and the right-hand side;
//  * columns are dealt to threads sorted by (x + y) parity, as in the z
//    march: every wavefront holds columns of one parity, so which plane of
//    each pair has the colour being updated is uniform over the wavefront,
//    and the register arrays take compile-time indices only;
//  * the columns' values are exchanged through LDS, plane-major and indexed
//    by the rank of the column in its class, so a half-sweep reads its
//    in-plane neighbours (the other class) at unit stride; a half-sweep
//    reads only the other colour and writes only its own, so one barrier per
//    half-sweep separates them;
//  * after NS half-sweeps the output columns (H inside the tile) and planes
//    (HZ inside the chunk) are exact: the halo is recomputed, as in the z
//    march, and u goes to the other copy;
//  * with RES, the pass also forms uc = R u and rc = R (rhs - L u) on the
//    coarse level (Eqs. 3-4): the halo is one cell wider, so the neighbours of
//    the output cells are final too;
//  * with the FAS flag (load prologue), the pass first forms the FAS
//    right-hand side R res + L u of the level just restricted into (Eq. 4)
//    from the loaded chunk, and stores it and t = u on its output cells.
//
// Global levels only (no segments): the tile covers the domain, out-of-domain
// neighbours are the zeros of the Dirichlet boundary.
#pragma once
#include <utility>
#include "kernels_fused.hpp"

namespace fmg {

// f(integral_constant<2 K + B>) for K = 0, 1, ...: the planes of one colour
template <int B, class Fn, int... K>
__device__ inline void for_planes(Fn&& f, std::integer_sequence<int, K...>) {
  (f(std::integral_constant<int, 2 * K + B>{}), ...);
}

template <class T, int NS, int PRO, int RES, int ZC>
__global__ void __launch_bounds__(1024) k_smooth_cols(SmoothArgs<T> a) {
  constexpr int NT = 1024, HZ = NS + RES, Z = ZC + 2 * HZ, H = NS + RES;
  static_assert(!RES || PRO == PRO_LOAD, "the epilogue follows a load prologue");
  static_assert(ZC % 2 == 0 && (PRO == PRO_LOAD || HZ % 2 == 0),
                "chunks of whole coarse planes; the prologues need an even first plane");
  // each column's chunk, plane-major
  __shared__ T ex[Z][NT];
  // epilogue: per-column sums over the two fine planes of each coarse plane
  __shared__ double lsu[RES ? ZC / 2 : 1][RES ? NT : 1], lsr[RES ? ZC / 2 : 1][RES ? NT : 1];

  const int n = a.gu.n, txw = a.txw, tyw = a.tyw, sx = txw - 2 * H, sy = tyw - 2 * H;
  // blocks are dealt round-robin to the L2 domains: give each domain a
  // contiguous range of tiles
  int tid = blockIdx.x;
  {
    const int nt = a.ntx * a.nty * a.ntz;
    const int per = udiv_fast(nt + a.nxcd - 1, a.nxcd);
    const int tq = udiv_fast(tid, a.nxcd);
    const int t2 = (tid - tq * a.nxcd) * per + tq;
    if (t2 >= nt) return;
    tid = t2;
  }
  const int tq1 = udiv_fast(tid, a.ntx), tk = udiv_fast(tq1, a.nty);
  const int ti = tid - tq1 * a.ntx, tj = tq1 - tk * a.nty;
  const int ox = ti * sx, oy = tj * sy, oz = tk * ZC, z0 = oz - HZ;
  // slots [0, NT/2) hold the columns of even (cx + cy), [NT/2, NT) the odd
  // ones (txw is even, so every row has txw/2 of each); a column's rank in
  // its class is i = cy txw/2 + cx/2.  Its x neighbours are in the other
  // class at ranks i - 1 + (cx & 1) and i + (cx & 1), its y neighbours at
  // ranks i -+ txw/2.  ox and oy are even, so the class is the parity of
  // x + y.
  const int t = threadIdx.x, tw2 = txw >> 1;
  const int hc = t >= NT / 2 ? 1 : 0, rk = t - hc * (NT / 2);
  // the same class, as a wavefront-uniform value (NT/2 is a multiple of 64)
  const int hw = __builtin_amdgcn_readfirstlane(t) >= NT / 2 ? 1 : 0;
  const bool col = rk < tw2 * tyw;
  const int cy = col ? udiv_small(rk, tw2) : 0;  // tw2 <= 128
  const int cx = col ? 2 * (rk - cy * tw2) + ((cy + hc) & 1) : 0;
  const int x = ox - H + cx, y = oy - H + cy;
  const bool st = col && x >= 0 && x < n && y >= 0 && y < n;
  // updated: inside the domain and not on the tile's edge
  const bool act = st && cx > 0 && cx < txw - 1 && cy > 0 && cy < tyw - 1;
  const bool outc = st && cx >= H && cx < txw - H && cy >= H && cy < tyw - H;
  // neighbour reads in the other class: around the column's rank, or around
  // rank txw/2 for columns never updated, so that every read is in bounds
  const int oc = hc ? 0 : NT / 2;  // the other class's slots
  const int ir = act ? rk : tw2;
  const int xn = oc + ir - 1 + (cx & 1), yn = oc + ir - tw2, yp = oc + ir + tw2;
  const int nbxy = (x == 0) + (x == n - 1) + (y == 0) + (y == n - 1);
  // the column's diagonal inverse 1 / (6 + boundary faces) off a z wall and on
  // one (the levels here have edges of at least 2, so no cell touches both)
  const T inv0 = (T)1 / (T)(6 + nbxy), inv1 = (T)1 / (T)(7 + nbxy);
  const Box B = seg_box_d(a.gu, 0), Br = seg_box_d(a.gr, 0);
  const long long pu = st ? at(a.gu, B, x, y, 0) : 0, pr = st ? at(a.gr, Br, x, y, 0) : 0;
  const long long mu = (long long)a.gu.m * a.gu.m, mr = (long long)a.gr.m * a.gr.m;

  // the chunk: every load issued before the first use.  Lanes with nothing to
  // read fetch element 0; their values are masked.
  T U[Z], F[Z];
#pragma unroll
  for (int j = 0; j < Z; ++j) {
    const int z = z0 + j;
    const bool v = st && z >= 0 && z < n;
    if (PRO != PRO_INTERP) U[j] = a.uin[v ? pu + z * mu : 0];
    F[j] = a.rhs[v ? pr + z * mr : 0];
  }
  if constexpr (PRO == PRO_CORRECT) {
    // u + (w - t) of the parent (Eq. 4's correction, piecewise constant):
    // fine planes 2K, 2K + 1 of the chunk share parent plane z0 / 2 + K
    const Box Bc = seg_box_d(a.gc, 0);
    const int nc = a.gc.n;
    const long long pc = st ? at(a.gc, Bc, x >> 1, y >> 1, 0) : 0;
    const long long mc = (long long)a.gc.m * a.gc.m;
    T W[Z / 2], Tt[Z / 2];
#pragma unroll
    for (int k = 0; k < Z / 2; ++k) {
      const int P = (z0 >> 1) + k;
      const bool v = st && P >= 0 && P < nc;
      W[k] = a.c[v ? pc + P * mc : 0];
      Tt[k] = a.ct[v ? pc + P * mc : 0];
    }
#pragma unroll
    for (int j = 0; j < Z; ++j) {
      const int z = z0 + j;
      const bool v = st && z >= 0 && z < n;
      U[j] = v ? U[j] + (W[j >> 1] - Tt[j >> 1]) : (T)0;
    }
  } else if constexpr (PRO == PRO_INTERP) {
    // FMG interpolation: trilinear, odd reflection at the walls.  The coarse
    // columns (X0, Y0), (X1, Y0), (X0, Y1), (X1, Y1) with X1 the next (odd x)
    // or previous coarse column; a column past the wall is X0 with sign -1.
    // Coarse planes z0 / 2 - 1 + K, K = 0 .. Z / 2 + 1, reflected likewise.
    const Box Bc = seg_box_d(a.gc, 0);
    const int nc = a.gc.n;
    const int X0 = x >> 1, Y0 = y >> 1;
    int X1 = (x & 1) ? X0 + 1 : X0 - 1, Y1 = (y & 1) ? Y0 + 1 : Y0 - 1;
    const bool rx = X1 < 0 || X1 >= nc, ry = Y1 < 0 || Y1 >= nc;
    X1 = rx ? X0 : X1;
    Y1 = ry ? Y0 : Y1;
    const long long mc = (long long)a.gc.m * a.gc.m;
    const long long q00 = st ? at(a.gc, Bc, X0, Y0, 0) : 0, q10 = st ? at(a.gc, Bc, X1, Y0, 0) : 0;
    const long long q01 = st ? at(a.gc, Bc, X0, Y1, 0) : 0, q11 = st ? at(a.gc, Bc, X1, Y1, 0) : 0;
    constexpr int NK = Z / 2 + 2;
    T C0[NK], C1[NK], C2[NK], C3[NK];
#pragma unroll
    for (int k = 0; k < NK; ++k) {
      int P = (z0 >> 1) - 1 + k;
      P = P < 0 ? -1 - P : (P >= nc ? 2 * nc - 1 - P : P);
      const bool v = st && P >= 0 && P < nc;
      C0[k] = a.c[v ? q00 + P * mc : 0];
      C1[k] = a.c[v ? q10 + P * mc : 0];
      C2[k] = a.c[v ? q01 + P * mc : 0];
      C3[k] = a.c[v ? q11 + P * mc : 0];
    }
    T cp[NK];  // xy interpolation on each coarse plane (weights 9, 3, 3, 1 / 16)
#pragma unroll
    for (int k = 0; k < NK; ++k) {
      const int P = (z0 >> 1) - 1 + k;
      const bool flip = P < 0 || P >= nc;
      const T s1 = rx ? -C1[k] : C1[k];
      const T s2 = ry ? -C2[k] : C2[k];
      const T s3 = (rx != ry) ? -C3[k] : C3[k];
      const T c = (T)0.5625 * C0[k] + ((T)0.1875 * (s1 + s2) + (T)0.0625 * s3);
      cp[k] = flip ? -c : c;
    }
    // fine plane z0 + j: 3/4 of its own coarse plane, 1/4 of the next (odd
    // z) or previous one
#pragma unroll
    for (int j = 0; j < Z; ++j) {
      const int z = z0 + j;
      const bool v = st && z >= 0 && z < n;
      const T cn = cp[(j >> 1) + 1], cf = cp[(j >> 1) + ((j & 1) ? 2 : 0)];
      U[j] = v ? (T)0.75 * cn + (T)0.25 * cf : (T)0;
    }
  } else {
#pragma unroll
    for (int j = 0; j < Z; ++j) {
      const int z = z0 + j;
      U[j] = (st && z >= 0 && z < n) ? U[j] : (T)0;
    }
  }
#pragma unroll
  for (int j = 0; j < Z; ++j) F[j] = (st && z0 + j >= 0 && z0 + j < n) ? F[j] : (T)0;
#pragma unroll
  for (int j = 0; j < Z; ++j) ex[j][t] = U[j];
  __syncthreads();

  if (PRO == PRO_LOAD && a.fas) {
    // rhs = R res + L u (FP64, neighbours summed in the order of the
    // single-cell kernels; out-of-domain neighbours are the zeros loaded)
    const double s2 = (double)n * (double)n;
#pragma unroll
    for (int j = 1; j < Z - 1; ++j) {
      const int z = z0 + j;
      const T* pl = ex[j];
      double sn = (double)pl[xn];
      sn += (double)pl[xn + 1];
      sn += (double)pl[yn];
      sn += (double)pl[yp];
      sn += (double)U[j - 1];
      sn += (double)U[j + 1];
      const double nb = (double)(6 + nbxy + (z == 0) + (z == n - 1));
      const double Lu = (sn - nb * (double)U[j]) * s2;
      const bool v = act && z >= 0 && z < n;
      F[j] = v ? (T)((double)F[j] + Lu) : F[j];
      if (v && outc && j >= HZ && j < HZ + ZC) {
        a.rhsw[pr + z * mr] = F[j];
        a.tw[pu + z * mu] = U[j];
      }
    }
    __syncthreads();  // the loaded values were read before the first half-sweep writes
  }

  // half-sweep s updates colour (s - 1) & 1, red ((x + y + z) even) first.
  // Of planes 2k and 2k + 1 the column's cell of that colour is plane
  // 2k + b, b = (x + y + z0 + colour) & 1, the same for the whole wavefront.
  // The chunk's first and last planes are never updated (their z neighbours
  // lie outside the chunk).
  auto cell = [&](auto jc) {
    constexpr int j = decltype(jc)::value;
    const int z = z0 + j;
    const T* pl = ex[j];
    const T below = j > 0 ? U[j > 0 ? j - 1 : 0] : (T)0;
    const T above = j < Z - 1 ? U[j < Z - 1 ? j + 1 : 0] : (T)0;
    const T sum = (((pl[xn] + pl[xn + 1]) + (pl[yn] + pl[yp])) + below) + above;
    const T inv = (z == 0 || z == n - 1) ? inv1 : inv0;
    const T nv = (sum - a.h2 * F[j]) * inv;
    const bool upd = act && j > 0 && j < Z - 1 && z >= 0 && z < n;
    U[j] = upd ? nv : U[j];
    if (upd) ex[j][t] = nv;
  };
#pragma unroll
  for (int s = 1; s <= NS; ++s) {
    if ((hw + z0 + ((s - 1) & 1)) & 1) for_planes<1>(cell, std::make_integer_sequence<int, Z / 2>{});
    else for_planes<0>(cell, std::make_integer_sequence<int, Z / 2>{});
    __syncthreads();
  }

  // the output planes of the output columns to the other copy
#pragma unroll
  for (int j = HZ; j < HZ + ZC; ++j) {
    const int z = z0 + j;
    if (outc && z < n) a.u[pu + z * mu] = U[j];
  }

  if constexpr (RES) {
    // residual of the output cells (Eq. 3; in FP64), summed over the two
    // fine planes of each coarse plane, then over the 2 x 2 columns of each
    // coarse cell by the column holding child (0, 0)
    const double s2 = (double)n * (double)n;
#pragma unroll
    for (int k = 0; k < ZC / 2; ++k) {
      double su = 0.0, sr = 0.0;
#pragma unroll
      for (int jj = 0; jj < 2; ++jj) {
        const int j = HZ + 2 * k + jj, z = z0 + j;
        const T* pl = ex[j];
        const double sn = (((double)pl[xn] + (double)pl[xn + 1]) +
                           ((double)pl[yn] + (double)pl[yp])) +
                          ((double)U[j - 1] + (double)U[j + 1]);
        const double uv = (double)U[j];
        const double nb = (double)(6 + nbxy + (z == 0) + (z == n - 1));
        su += uv;
        sr += (double)F[j] - (sn - nb * uv) * s2;
      }
      if (outc) {
        lsu[k][t] = su;
        lsr[k][t] = sr;
      }
    }
    __syncthreads();
    // (the output region starts on even x and y and has even extent, so the
    // 2 x 2 columns are output columns): this slot, the other class at ranks
    // + (cx & 1) and + txw/2, and this class at rank + txw/2 + (cx & 1)
    const bool own = outc && (x & 1) == 0 && (y & 1) == 0;
    const int od = cx & 1, pn = oc + rk;
    if (own) {
      const Box Bo = seg_box_d(a.gcr, 0);
#pragma unroll
      for (int k = 0; k < ZC / 2; ++k) {
        const int Zc = (oz >> 1) + k;
        if (2 * Zc >= n) break;
        const double tu = (lsu[k][t] + lsu[k][pn + od]) + (lsu[k][pn + tw2] + lsu[k][t + tw2 + od]);
        const double tr = (lsr[k][t] + lsr[k][pn + od]) + (lsr[k][pn + tw2] + lsr[k][t + tw2 + od]);
        const long long id = at(a.gcr, Bo, x >> 1, y >> 1, Zc);
        a.uc[id] = (T)(tu / 8.0);
        a.rc[id] = (T)(tr / 8.0);
      }
    }
  }
}

}  // namespace fmg
