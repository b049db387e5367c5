// fv27.hip -- FAS full multigrid with segmental refinement for the paper's
// own model problem (Sec. 5.1 of "Segmental Refinement: A Multigrid Technique
// for Data Locality", arXiv:1406.7808) on gfx950: a box of cubic cells, the
// 27-point finite volume Laplacian, Chebyshev smoothers, trilinear
// prolongation for both the FMG and the V-cycle, segments as an s0 x s1 x s2
// array of cubic subdomains (the paper's process grid).
//
// The operator has tensor-product form: L = h^-2 (D2_x W_y W_z + W_x D2_y W_z
// + W_x W_y D2_z) with D2 = (1, -2, 1) and the face-average weights
// W = (w1, w0, w1) = (1/24, 11/12, 1/24).  Grouping by z gives
//   L u(z) = h^-2 [ W_z P + D2_z Q ](z),
//   P = (D2_x W_y + W_x D2_y) u,  Q = W_x W_y u   (9-point, in one xy plane),
// so the smoothing kernel marches an xy tile through z, forms P and Q of each
// plane from the plane staged in LDS (9 reads give both), keeps the last
// three planes' P and Q in registers and combines them: 9 LDS reads per cell
// instead of 27.  A ghost beyond a wall is the odd reflection of the interior
// cell, per dimension, so a plane beyond a z wall is minus its mirror and
// its P and Q are minus the mirror's.
//
// Storage: a global level is one n0 x n1 x n2 array (x fastest).  An SR
// level holds one box per segment covering its compute region C and one
// ghost layer (the frozen GSR cells inside the domain); box q sits at q * box
// with fixed extents m[d] = min(n[d], g + 2J) + 2 (boxes of clipped segments
// leave their tail unused).  Each level has two copies of u: a Chebyshev
// step is a Jacobi-type update and reads one copy while writing the other on
// C.  Ghost cells change only under prolongation, which writes both copies.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/fmg.h"
#include "../../include/fv27.h"

namespace fv {

constexpr double kW0 = 11.0 / 12.0;
constexpr double kW1 = 1.0 / 24.0;
constexpr int kTX = 32, kTY = 8, kThreads = kTX * kTY;  // march tile
constexpr int kBlock = 256;                              // per-cell kernels
constexpr int kMaxCoarse = 512;                          // cells of the coarsest level

static thread_local std::string g_err;

static int32_t fail(int32_t st, const std::string& msg) {
  g_err = msg;
  return st;
}

struct hip_error {
  std::string what;
};

static void hipcheck(hipError_t e, const char* what) {
  if (e != hipSuccess) throw hip_error{std::string(what) + ": " + hipGetErrorString(e)};
}

// ---------------------------------------------------------------------------
// level geometry
// ---------------------------------------------------------------------------

struct Geo {
  int n[3];       // level extents
  int S[3];       // segments per dimension (1,1,1 for a global level)
  int g;          // genuine edge of a segment (cubic)
  int J;          // buffer width
  int m[3];       // storage extents of one box
  int sr;         // 1: segment boxes with a ghost layer; 0: one global array
  long long box;  // cells of one box
};

static Geo global_geo(const int n[3]) {
  Geo G;
  for (int d = 0; d < 3; ++d) {
    G.n[d] = n[d];
    G.S[d] = 1;
    G.m[d] = n[d];
  }
  G.g = 0;
  G.J = 0;
  G.sr = 0;
  G.box = (long long)n[0] * n[1] * n[2];
  return G;
}

static Geo seg_geo(const int n[3], const int S[3], int J) {
  Geo G;
  G.g = n[0] / S[0];
  for (int d = 0; d < 3; ++d) {
    G.n[d] = n[d];
    G.S[d] = S[d];
    G.m[d] = std::min(n[d], G.g + 2 * J) + 2;
  }
  G.J = J;
  G.sr = 1;
  G.box = (long long)G.m[0] * G.m[1] * G.m[2];
  return G;
}

static int nseg(const Geo& G) { return G.S[0] * G.S[1] * G.S[2]; }

// compute region [clo, chi) and storage origin slo of segment q
__host__ __device__ inline void seg_region(const Geo& G, int q, int clo[3], int chi[3],
                                           int slo[3]) {
  int p[3] = {q % G.S[0], (q / G.S[0]) % G.S[1], q / (G.S[0] * G.S[1])};
  for (int d = 0; d < 3; ++d) {
    if (G.sr) {
      int a = p[d] * G.g - G.J, b = (p[d] + 1) * G.g + G.J;
      clo[d] = a < 0 ? 0 : a;
      chi[d] = b > G.n[d] ? G.n[d] : b;
      slo[d] = clo[d] - 1;
    } else {
      clo[d] = 0;
      chi[d] = G.n[d];
      slo[d] = 0;
    }
  }
}

// genuine region of segment q
__host__ __device__ inline void seg_genuine(const Geo& G, int q, int vlo[3], int vhi[3]) {
  int p[3] = {q % G.S[0], (q / G.S[0]) % G.S[1], q / (G.S[0] * G.S[1])};
  for (int d = 0; d < 3; ++d) {
    int e = G.n[d] / G.S[d];
    vlo[d] = p[d] * e;
    vhi[d] = (p[d] + 1) * e;
  }
}

__host__ __device__ inline long long sidx(const Geo& G, int q, const int slo[3], int x, int y,
                                          int z) {
  return (long long)q * G.box +
         ((long long)(z - slo[2]) * G.m[1] + (y - slo[1])) * G.m[0] + (x - slo[0]);
}

// odd reflection of one index into [0, n); returns the sign
__device__ inline double mirror(int n, int& i) {
  if (i < 0) {
    i = -1 - i;
    return -1.0;
  }
  if (i >= n) {
    i = 2 * n - 1 - i;
    return -1.0;
  }
  return 1.0;
}

// value of cell (x,y,z) of level storage v (segment q), ghosts beyond a wall
// by odd reflection
template <class T>
__device__ inline double value(const T* v, const Geo& G, int q, const int slo[3], int x, int y,
                               int z) {
  double s = mirror(G.n[0], x) * mirror(G.n[1], y) * mirror(G.n[2], z);
  return s * (double)v[sidx(G, q, slo, x, y, z)];
}

// 27-point L v at cell (x,y,z), read directly (per-cell kernels on small or
// coarse levels); same grouping as the march: W_z P + D2_z Q
__device__ inline double apply_L_direct(const double* v, const Geo& G, int q, const int slo[3],
                                        int x, int y, int z, double inv_h2) {
  double P[3], Q[3];
  for (int c = 0; c < 3; ++c) {
    double a[3][3];
    for (int b = 0; b < 3; ++b)
      for (int e = 0; e < 3; ++e) a[b][e] = value(v, G, q, slo, x + e - 1, y + b - 1, z + c - 1);
    const double ctr = a[1][1];
    const double face = (a[1][0] + a[1][2]) + (a[0][1] + a[2][1]);
    const double corner = (a[0][0] + a[0][2]) + (a[2][0] + a[2][2]);
    P[c] = -4.0 * kW0 * ctr + (kW0 - 2.0 * kW1) * face + 2.0 * kW1 * corner;
    Q[c] = kW0 * kW0 * ctr + kW0 * kW1 * face + kW1 * kW1 * corner;
  }
  return (kW1 * (P[0] + P[2]) + kW0 * P[1] + (Q[0] + Q[2]) - 2.0 * Q[1]) * inv_h2;
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

struct MarchArgs {
  Geo G;
  const double* u;    // input copy
  double* out;        // output copy (Chebyshev step) or residual array
  const double* rhs;  // right-hand side: level storage, or a global array
  int rhs_global;     // rhs indexed as a global n0 x n1 x n2 array
  int mode;           // 0: out = u - c (rhs - L u) on C; 1: out = rhs - L u on C;
                      // 2: out = L u on C (rhs unused)
  double c;
  double inv_h2;
  int tiles_x, zchunk;
  double* fin;  // the solve's last step: genuine cells also go to the caller's u (or null)
};

// An xy tile of kTX x kTY columns of one segment's compute region marches a
// z chunk.  Each step stages one plane of u (tile + 1-cell halo, ghosts and
// reflections resolved) in LDS, forms that plane's P and Q, and finishes the
// plane one below.  Double-buffered planes: one barrier per step.  Each
// thread's staged cells keep their column offset and reflection sign from
// the start, and their values (and the right-hand side of the next output
// cell) are loaded one step ahead, so the loads of a plane are in flight
// while the step before it computes.
__global__ void __launch_bounds__(kThreads) k_fv_march(MarchArgs A) {
  const Geo& G = A.G;
  const int q = blockIdx.z;
  int clo[3], chi[3], slo[3];
  seg_region(G, q, clo, chi, slo);
  const int tx = blockIdx.x % A.tiles_x, ty = blockIdx.x / A.tiles_x;
  const int x0 = clo[0] + tx * kTX, y0 = clo[1] + ty * kTY;
  const int z0 = clo[2] + blockIdx.y * A.zchunk;
  if (x0 >= chi[0] || y0 >= chi[1] || z0 >= chi[2]) return;  // uniform over the block
  const int z1 = min(chi[2], z0 + A.zchunk);
  const int lx = threadIdx.x % kTX, ly = threadIdx.x / kTX;
  const int x = x0 + lx, y = y0 + ly;
  const bool active = x < chi[0] && y < chi[1];
  // halo columns beyond C + 1 are never needed (and lie outside the box)
  const int xh = min(x0 + kTX, chi[0]), yh = min(y0 + kTY, chi[1]);

  // staged cells of this thread: LDS place, storage offset of the column in
  // plane slo[2], reflection sign in x and y (0: not staged, stores 0)
  constexpr int kPl = (kTX + 2) * (kTY + 2), kSl = (kPl + kThreads - 1) / kThreads;
  int sp[kSl];
  long long so[kSl];
  double ss[kSl];
#pragma unroll
  for (int k = 0; k < kSl; ++k) {
    const int i = threadIdx.x + k * kThreads;
    sp[k] = i;
    so[k] = (long long)q * G.box;
    ss[k] = 0.0;
    if (i < kPl) {
      int gx = x0 - 1 + i % (kTX + 2), gy = y0 - 1 + i / (kTX + 2);
      if (gx <= xh && gy <= yh) {
        const double sx = mirror(G.n[0], gx), sy = mirror(G.n[1], gy);
        ss[k] = sx * sy;
        so[k] += (long long)(gy - slo[1]) * G.m[0] + (gx - slo[0]);
      }
    }
  }
  const long long pm = (long long)G.m[0] * G.m[1];
  // values of the staged cells in plane zl
  auto fetch = [&](int zl, double(&v)[kSl]) {
    const double sz = mirror(G.n[2], zl);
    const long long oz = (long long)(zl - slo[2]) * pm;
#pragma unroll
    for (int k = 0; k < kSl; ++k) {
      const double w = A.u[so[k] + oz];
      v[k] = ss[k] != 0.0 ? (ss[k] * sz) * w : 0.0;
    }
  };
  // right-hand side of this thread's cell in plane zc
  const bool wants_f = active && A.mode != 2;
  auto fetch_f = [&](int zc) -> double {
    return A.rhs_global ? A.rhs[((long long)zc * G.n[1] + y) * G.n[0] + x]
                        : A.rhs[sidx(G, q, slo, x, y, zc)];
  };

  __shared__ double plane[2][kTY + 2][kTX + 2];
  double P0 = 0, P1 = 0, P2 = 0, Q0 = 0, Q1 = 0, Q2 = 0, c1 = 0, c2 = 0;
  const int nsteps = z1 - z0 + 2;
  double va[kSl], vb[kSl];
  double fa = 0.0, fb = 0.0;  // right-hand side of this step's and the next step's output cell
  fetch(z0 - 1, va);
  for (int s = 0; s < nsteps; ++s) {
    const int zl = z0 - 1 + s;
    double(*pl)[kTX + 2] = plane[s & 1];
#pragma unroll
    for (int k = 0; k < kSl; ++k)
      if (sp[k] < kPl) (&pl[0][0])[sp[k]] = va[k];
    if (s + 1 < nsteps) {
      fetch(zl + 1, vb);
      if (s >= 1 && wants_f) fb = fetch_f(zl);  // step s + 1 finishes plane zl
    }
    __syncthreads();
    const double ctr = pl[ly + 1][lx + 1];
    const double face = (pl[ly + 1][lx] + pl[ly + 1][lx + 2]) + (pl[ly][lx + 1] + pl[ly + 2][lx + 1]);
    const double corner = (pl[ly][lx] + pl[ly][lx + 2]) + (pl[ly + 2][lx] + pl[ly + 2][lx + 2]);
    P0 = P1;
    P1 = P2;
    P2 = -4.0 * kW0 * ctr + (kW0 - 2.0 * kW1) * face + 2.0 * kW1 * corner;
    Q0 = Q1;
    Q1 = Q2;
    Q2 = kW0 * kW0 * ctr + kW0 * kW1 * face + kW1 * kW1 * corner;
    c1 = c2;
    c2 = ctr;
    if (s >= 2 && active) {
      const int zc = zl - 1;
      const double Lu = (kW1 * (P0 + P2) + kW0 * P1 + (Q0 + Q2) - 2.0 * Q1) * A.inv_h2;
      const long long id = sidx(G, q, slo, x, y, zc);
      if (A.mode == 2) {
        A.out[id] = Lu;
      } else {
        const double r = fa - Lu;
        const double v = A.mode ? r : c1 - A.c * r;
        A.out[id] = v;
        if (A.fin) {  // the genuine cells of the finest level (every cell of a global one)
          int vlo[3], vhi[3];
          seg_genuine(G, q, vlo, vhi);
          if (x >= vlo[0] && x < vhi[0] && y >= vlo[1] && y < vhi[1] && zc >= vlo[2] && zc < vhi[2])
            A.fin[((long long)zc * G.n[1] + y) * G.n[0] + x] = v;
        }
      }
    }
#pragma unroll
    for (int k = 0; k < kSl; ++k) va[k] = vb[k];
    fa = fb;
  }
}

// Two Chebyshev steps in one pass (temporal blocking): u1 = u - c (rhs - L u)
// and u2 = u1 - c2 (rhs - L u1) on C.  The tile's planes of u are staged with
// a 2-cell halo; stage 1 forms u1 on the tile plus a 1-cell halo, one plane
// behind the load, into a second LDS plane; stage 2 forms u2 on the tile, one
// plane behind stage 1.  u1 is u itself on the frozen ghosts; beyond a wall
// stage 2 reads u1 by reflection (mirrored LDS index in x and y, negated P
// and Q of the wall plane in z), so stage 1 computes only inside the domain.
constexpr int kT2X = kTX + 2, kT2Y = kTY + 2;          // stage-1 region
constexpr int kThreads2 = 512;                          // >= kT2X * kT2Y
static_assert(kT2X * kT2Y <= kThreads2, "stage 1 needs one thread per column");

__global__ void __launch_bounds__(kThreads2) k_fv_march2(MarchArgs A, double c2) {
  const Geo& G = A.G;
  const int q = blockIdx.z;
  int clo[3], chi[3], slo[3];
  seg_region(G, q, clo, chi, slo);
  const int tx = blockIdx.x % A.tiles_x, ty = blockIdx.x / A.tiles_x;
  const int x0 = clo[0] + tx * kTX, y0 = clo[1] + ty * kTY;
  const int z0 = clo[2] + blockIdx.y * A.zchunk;
  if (x0 >= chi[0] || y0 >= chi[1] || z0 >= chi[2]) return;  // uniform over the block
  const int z1 = min(chi[2], z0 + A.zchunk);
  const int nz = G.n[2];

  __shared__ double U0[2][kTY + 4][kTX + 4];
  __shared__ double U1[2][kT2Y][kT2X];

  // stage 1: column (c1x, c1y) of the tile plus a 1-cell halo
  const int tid = threadIdx.x;
  const bool s1 = tid < kT2X * kT2Y;
  const int c1x = tid % kT2X, c1y = tid / kT2X;
  const int x1 = x0 - 1 + c1x, y1 = y0 - 1 + c1y;
  const bool dom1 = x1 >= 0 && x1 < G.n[0] && y1 >= 0 && y1 < G.n[1];
  const bool inc1 = x1 >= clo[0] && x1 < chi[0] && y1 >= clo[1] && y1 < chi[1];
  const bool sto1 = x1 >= clo[0] - 1 && x1 <= chi[0] && y1 >= clo[1] - 1 && y1 <= chi[1];
  // stage 2: column (c2x, c2y) of the tile; its 3 x 3 neighbours in U1, a
  // neighbour beyond a wall read at its mirror with the sign -1
  const bool s2 = tid < kTX * kTY;
  const int c2x = tid % kTX, c2y = tid / kTX;
  const int x2 = x0 + c2x, y2 = y0 + c2y;
  const bool act2 = s2 && x2 < chi[0] && y2 < chi[1];
  int ix[3], iy[3];
  double sx[3], sy[3];
  for (int k = 0; k < 3; ++k) {
    int gx = x2 + k - 1, gy = y2 + k - 1;
    sx[k] = mirror(G.n[0], gx);
    sy[k] = mirror(G.n[1], gy);
    // (inactive columns may map outside the plane: clamp, they store nothing)
    ix[k] = min(max(gx - (x0 - 1), 0), kT2X - 1);
    iy[k] = min(max(gy - (y0 - 1), 0), kT2Y - 1);
  }
  // positions more than two cells from C are never needed; those within,
  // inside the domain, must lie in the box (C and its ghost layer), and those
  // beyond a wall mirror into C
  auto loadable = [&](int g, int d) {
    return g >= clo[d] - 2 && g <= chi[d] + 1 &&
           (g < 0 || g >= G.n[d] || (g >= clo[d] - 1 && g <= chi[d]));
  };

  // the staged cell of this thread (one per thread: (kTX + 4)(kTY + 4) <=
  // kThreads2): storage offset of its column in plane slo[2] and reflection
  // sign in x and y (0: not loaded); values and right-hand sides are loaded
  // one step ahead, as in k_fv_march
  static_assert((kTX + 4) * (kTY + 4) <= kThreads2, "one staged cell per thread");
  const bool st0 = tid < (kTX + 4) * (kTY + 4);
  long long so = (long long)q * G.box;
  double ss = 0.0;
  if (st0) {
    int gx = x0 - 2 + tid % (kTX + 4), gy = y0 - 2 + tid / (kTX + 4);
    if (loadable(gx, 0) && loadable(gy, 1)) {
      const double sgx = mirror(G.n[0], gx), sgy = mirror(G.n[1], gy);
      ss = sgx * sgy;
      so += (long long)(gy - slo[1]) * G.m[0] + (gx - slo[0]);
    }
  }
  const long long pm = (long long)G.m[0] * G.m[1];
  auto fetch = [&](int zl) -> double {
    if (!loadable(zl, 2)) return 0.0;  // uniform over the block
    const double sz = mirror(G.n[2], zl);
    const double w = A.u[so + (long long)(zl - slo[2]) * pm];
    return ss != 0.0 ? (ss * sz) * w : 0.0;
  };
  auto rhs_at = [&](int x, int y, int z) -> double {
    return A.rhs_global ? A.rhs[((long long)z * G.n[1] + y) * G.n[0] + x]
                        : A.rhs[sidx(G, q, slo, x, y, z)];
  };
  // stage 1 forms u1 of plane zo1 on its column, stage 2 u2 of plane zo2
  auto f1_wanted = [&](int zo1) {
    return s1 && zo1 >= 0 && zo1 < nz && dom1 && inc1 && zo1 >= clo[2] && zo1 < chi[2];
  };
  auto f2_wanted = [&](int zo2) { return act2 && zo2 >= z0 && zo2 < z1; };

  double P0 = 0, P1 = 0, P2 = 0, Q0 = 0, Q1 = 0, Q2 = 0, cA = 0, cB = 0;  // stage 1 window
  double R0 = 0, R1 = 0, R2 = 0, S0 = 0, S1 = 0, S2 = 0, dA = 0, dB = 0;  // stage 2 window
  const int nsteps = z1 - z0 + 4;  // u planes z0 - 2 .. z1 + 1
  double va = fetch(z0 - 2), vb = 0.0;
  double f1a = 0.0, f1b = 0.0, f2a = 0.0, f2b = 0.0;  // right-hand sides, this step and the next
  for (int s = 0; s < nsteps; ++s) {
    const int zl = z0 - 2 + s;
    double(*u0)[kTX + 4] = U0[s & 1];
    double(*u1)[kT2X] = U1[s & 1];
    if (st0) (&u0[0][0])[tid] = va;
    if (s + 1 < nsteps) {  // step s + 1: plane zl + 1, stage 1 at zl, stage 2 at zl - 1
      vb = fetch(zl + 1);
      if (s + 1 >= 2 && f1_wanted(zl)) f1b = rhs_at(x1, y1, zl);
      if (s + 1 >= 2 && f2_wanted(zl - 1)) f2b = rhs_at(x2, y2, zl - 1);
    }
    __syncthreads();
    // stage 1: P and Q of plane zl; u1 of plane zl - 1
    const int zo1 = zl - 1;
    if (s1) {
      const int lx = c1x + 1, ly = c1y + 1;
      const double ctr = u0[ly][lx];
      const double face = (u0[ly][lx - 1] + u0[ly][lx + 1]) + (u0[ly - 1][lx] + u0[ly + 1][lx]);
      const double corner =
          (u0[ly - 1][lx - 1] + u0[ly - 1][lx + 1]) + (u0[ly + 1][lx - 1] + u0[ly + 1][lx + 1]);
      P0 = P1;
      P1 = P2;
      P2 = -4.0 * kW0 * ctr + (kW0 - 2.0 * kW1) * face + 2.0 * kW1 * corner;
      Q0 = Q1;
      Q1 = Q2;
      Q2 = kW0 * kW0 * ctr + kW0 * kW1 * face + kW1 * kW1 * corner;
      cA = cB;
      cB = ctr;
      if (s >= 2 && zo1 >= 0 && zo1 < nz) {
        double v = 0.0;
        const bool inz = zo1 >= clo[2] && zo1 < chi[2];
        if (dom1 && inc1 && inz) {
          const double Lu = (kW1 * (P0 + P2) + kW0 * P1 + (Q0 + Q2) - 2.0 * Q1) * A.inv_h2;
          v = cA - A.c * (f1a - Lu);
        } else if (dom1 && sto1 && zo1 >= clo[2] - 1 && zo1 <= chi[2]) {
          v = cA;  // a frozen ghost: u1 = u
        }
        u1[c1y][c1x] = v;
      }
    }
    __syncthreads();
    // stage 2: P and Q of u1's plane zo1 (its mirror beyond a z wall); u2 of
    // plane zo1 - 1
    if (s >= 2 && zo1 >= -1 && zo1 <= nz && s2) {
      double Pn, Qn, ctr = 0.0;
      if (zo1 >= 0 && zo1 < nz) {
        double a[3][3];
        for (int b = 0; b < 3; ++b)
          for (int e = 0; e < 3; ++e) a[b][e] = sx[e] * sy[b] * u1[iy[b]][ix[e]];
        ctr = a[1][1];
        const double face = (a[1][0] + a[1][2]) + (a[0][1] + a[2][1]);
        const double corner = (a[0][0] + a[0][2]) + (a[2][0] + a[2][2]);
        Pn = -4.0 * kW0 * ctr + (kW0 - 2.0 * kW1) * face + 2.0 * kW1 * corner;
        Qn = kW0 * kW0 * ctr + kW0 * kW1 * face + kW1 * kW1 * corner;
      } else {  // plane -1 or nz: minus its mirror (0 or nz - 1)
        Pn = -R2;
        Qn = -S2;
      }
      if (zo1 >= -1 && !(zo1 == -1)) {
        R0 = R1;
        R1 = R2;
        R2 = Pn;
        S0 = S1;
        S1 = S2;
        S2 = Qn;
        dA = dB;
        dB = ctr;
        if (zo1 == 0) {  // the plane below the domain mirrors plane 0
          R1 = -R2;
          S1 = -S2;
        }
      }
      const int zo2 = zo1 - 1;
      if (act2 && zo2 >= z0 && zo2 < z1) {
        const double Lu = (kW1 * (R0 + R2) + kW0 * R1 + (S0 + S2) - 2.0 * S1) * A.inv_h2;
        const long long id = sidx(G, q, slo, x2, y2, zo2);
        const double v = dA - c2 * (f2a - Lu);
        A.out[id] = v;
        if (A.fin) {
          int vlo[3], vhi[3];
          seg_genuine(G, q, vlo, vhi);
          if (x2 >= vlo[0] && x2 < vhi[0] && y2 >= vlo[1] && y2 < vhi[1] && zo2 >= vlo[2] &&
              zo2 < vhi[2])
            A.fin[((long long)zo2 * G.n[1] + y2) * G.n[0] + x2] = v;
        }
      }
    }
    va = vb;
    f1a = f1b;
    f2a = f2b;
  }
}

// mean of the 8 children of coarse cell (I,J,K) of fine storage v
__device__ inline double mean8(const double* v, const Geo& F, int q, const int slo[3], int I,
                               int J, int K) {
  double s = 0.0;
  for (int c = 0; c < 2; ++c)
    for (int b = 0; b < 2; ++b)
      for (int a = 0; a < 2; ++a) s += v[sidx(F, q, slo, 2 * I + a, 2 * J + b, 2 * K + c)];
  return s / 8.0;
}

struct RestrictArgs {
  Geo F, C;          // fine and coarse geometry
  const double* fu;  // fine u (or f)
  const double* fr;  // fine residual (null: restrict fu only)
  double* cu;        // coarse u (or f)
  double* cr;        // coarse restricted residual
  int target;        // 0: every coarse cell (global to global); 1: F = C_fine / 2 of
                     // each segment into its coarse box; 2: genuine coarse cells of
                     // each segment into the global coarse level (owner computes)
  int ex[3];         // extents of the per-segment index space
};

__global__ void __launch_bounds__(kBlock) k_fv_restrict(RestrictArgs A) {
  const int q = blockIdx.y;
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)A.ex[0] * A.ex[1] * A.ex[2]) return;
  int o[3] = {(int)(t % A.ex[0]), (int)((t / A.ex[0]) % A.ex[1]), (int)(t / ((long long)A.ex[0] * A.ex[1]))};
  int flo[3], fhi[3], fslo[3];
  seg_region(A.F, q, flo, fhi, fslo);
  int lo[3], hi[3];
  if (A.target == 1) {
    for (int d = 0; d < 3; ++d) {
      lo[d] = flo[d] / 2;
      hi[d] = fhi[d] / 2;
    }
  } else if (A.target == 2) {
    int vlo[3], vhi[3];
    seg_genuine(A.F, q, vlo, vhi);
    for (int d = 0; d < 3; ++d) {
      lo[d] = vlo[d] / 2;
      hi[d] = vhi[d] / 2;
    }
  } else {
    for (int d = 0; d < 3; ++d) {
      lo[d] = 0;
      hi[d] = A.C.n[d];
    }
  }
  const int I = lo[0] + o[0], J = lo[1] + o[1], K = lo[2] + o[2];
  if (I >= hi[0] || J >= hi[1] || K >= hi[2]) return;
  int clo[3], chi[3], cslo[3];
  seg_region(A.C, A.target == 1 ? q : 0, clo, chi, cslo);
  const long long cid = sidx(A.C, A.target == 1 ? q : 0, cslo, I, J, K);
  A.cu[cid] = mean8(A.fu, A.F, q, fslo, I, J, K);
  if (A.fr) A.cr[cid] = mean8(A.fr, A.F, q, fslo, I, J, K);
}

struct FasArgs {
  Geo C;             // coarse level
  Geo F;             // the finer level (for the region F = C_fine / 2)
  const double* u;   // coarse u (restricted on F)
  const double* rr;  // restricted residual (valid on F, or everywhere if global)
  double* rhs;       // coarse right-hand side (on C)
  double* t;         // copy of u (whole storage inside the domain)
  double inv_h2;
};

// rhs = (R res on F, 0 on C \ F) + L_c u on C; t = u on C and ghosts
__global__ void __launch_bounds__(kBlock) k_fv_fas(FasArgs A) {
  const int q = blockIdx.y;
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const Geo& G = A.C;
  if (t >= G.box) return;
  int clo[3], chi[3], slo[3];
  seg_region(G, q, clo, chi, slo);
  const int x = slo[0] + (int)(t % G.m[0]), y = slo[1] + (int)((t / G.m[0]) % G.m[1]),
            z = slo[2] + (int)(t / ((long long)G.m[0] * G.m[1]));
  if (x < 0 || y < 0 || z < 0 || x >= G.n[0] || y >= G.n[1] || z >= G.n[2]) return;
  if (x > chi[0] || y > chi[1] || z > chi[2]) return;  // beyond this segment's box
  const long long id = q * G.box + t;
  A.t[id] = A.u[id];
  if (x < clo[0] || y < clo[1] || z < clo[2] || x >= chi[0] || y >= chi[1] || z >= chi[2]) return;
  bool inF = true;
  if (G.sr) {
    int flo[3], fhi[3], fslo[3];
    seg_region(A.F, q, flo, fhi, fslo);
    inF = x >= flo[0] / 2 && x < fhi[0] / 2 && y >= flo[1] / 2 && y < fhi[1] / 2 &&
          z >= flo[2] / 2 && z < fhi[2] / 2;
  }
  const double Lu = apply_L_direct(A.u, G, q, slo, x, y, z, A.inv_h2);
  A.rhs[id] = (inF ? A.rr[id] : 0.0) + Lu;
}

struct ProlongArgs {
  Geo F, C;          // fine (target) and coarse (source) geometry
  int csrc_seg;      // 1: the coarse source is the same segment's box; 0: global
  const double* w;   // coarse source (u for the FMG step; w for the correction)
  const double* t;   // coarse t (correction only; null for the FMG step)
  double* u0;        // fine copies: the current one (every cell) and the other (ghosts)
  double* u1;
  int add;           // 0: u = P w; 1: u += P (w - t)
};

// trilinear prolongation onto every storage cell inside the domain (C and
// the frozen ghosts) of the current copy, and onto the ghosts of the other
// copy: the FMG step, or the V-cycle correction.  One thread
// per coarse parent writes its (up to) 8 children: the 3 x 3 x 3 coarse
// values they use (w - t, or u; only those a child needs, reflected at the
// walls) are loaded once.  Each child sums its 8 weighted values in the same
// order as a child-by-child evaluation.
__global__ void __launch_bounds__(kBlock) k_fv_prolong(ProlongArgs A) {
  const int q = blockIdx.y;
  const Geo& G = A.F;
  int clo[3], chi[3], slo[3];
  seg_region(G, q, clo, chi, slo);
  int flo[3], fhi[3], plo[3], pe[3];
  for (int d = 0; d < 3; ++d) {  // fine cells written: storage inside the domain
    flo[d] = G.sr ? max(0, clo[d] - 1) : 0;
    fhi[d] = G.sr ? min(G.n[d], chi[d] + 1) : G.n[d];
    plo[d] = flo[d] >> 1;
    pe[d] = ((fhi[d] - 1) >> 1) + 1 - plo[d];
  }
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)pe[0] * pe[1] * pe[2]) return;
  const int P[3] = {plo[0] + (int)(t % pe[0]), plo[1] + (int)((t / pe[0]) % pe[1]),
                    plo[2] + (int)(t / ((long long)pe[0] * pe[1]))};
  bool v0[3], v1[3];  // child 2P (v0) and 2P + 1 (v1) written, per dimension
  for (int d = 0; d < 3; ++d) {
    v0[d] = 2 * P[d] >= flo[d] && 2 * P[d] < fhi[d];
    v1[d] = 2 * P[d] + 1 >= flo[d] && 2 * P[d] + 1 < fhi[d];
  }
  const int cq = A.csrc_seg ? q : 0;
  int cclo[3], cchi[3], cslo[3];
  seg_region(A.C, cq, cclo, cchi, cslo);
  double cv[3][3][3];
  for (int dz = 0; dz < 3; ++dz)
    for (int dy = 0; dy < 3; ++dy)
      for (int dx = 0; dx < 3; ++dx) {
        const bool need = (dz != 0 || v0[2]) && (dz != 2 || v1[2]) && (dy != 0 || v0[1]) &&
                          (dy != 2 || v1[1]) && (dx != 0 || v0[0]) && (dx != 2 || v1[0]);
        double v = 0.0;
        if (need) {
          int a = P[0] + dx - 1, b = P[1] + dy - 1, c = P[2] + dz - 1;
          const double sg = mirror(A.C.n[0], a) * mirror(A.C.n[1], b) * mirror(A.C.n[2], c);
          const long long cid = sidx(A.C, cq, cslo, a, b, c);
          v = sg * (A.add ? A.w[cid] - A.t[cid] : A.w[cid]);
        }
        cv[dz][dy][dx] = v;
      }
  for (int kz = 0; kz < 2; ++kz)
    for (int ky = 0; ky < 2; ++ky)
      for (int kx = 0; kx < 2; ++kx) {
        if (!(kz ? v1[2] : v0[2]) || !(ky ? v1[1] : v0[1]) || !(kx ? v1[0] : v0[0])) continue;
        // the other neighbour of the parent, per dimension: toward the child
        const int ox = kx ? 2 : 0, oy = ky ? 2 : 0, oz = kz ? 2 : 0;
        double s = 0.0;
        for (int cz = 0; cz < 2; ++cz)
          for (int cy = 0; cy < 2; ++cy)
            for (int cx = 0; cx < 2; ++cx) {
              const double wt = (cx ? 0.25 : 0.75) * (cy ? 0.25 : 0.75) * (cz ? 0.25 : 0.75);
              s += wt * cv[cz ? oz : 1][cy ? oy : 1][cx ? ox : 1];
            }
        const int fx = 2 * P[0] + kx, fy = 2 * P[1] + ky, fz = 2 * P[2] + kz;
        const long long id = sidx(G, q, slo, fx, fy, fz);
        const double nv = A.add ? A.u0[id] + s : s;
        A.u0[id] = nv;
        // the other copy needs only the ghosts: its compute region is
        // rewritten by the next smoothing step before it is read
        if (fx < clo[0] || fx >= chi[0] || fy < clo[1] || fy >= chi[1] || fz < clo[2] ||
            fz >= chi[2])
          A.u1[id] = nv;
      }
}

// u = Ainv rhs on the coarsest level (one workgroup)
__global__ void __launch_bounds__(kBlock) k_fv_coarse(const double* __restrict__ Ainv, int m,
                                                     const double* __restrict__ rhs,
                                                     double* __restrict__ u0,
                                                     double* __restrict__ u1) {
  __shared__ double r[kMaxCoarse];
  for (int i = threadIdx.x; i < m; i += blockDim.x) r[i] = rhs[i];
  __syncthreads();
  for (int i = threadIdx.x; i < m; i += blockDim.x) {
    double s = 0.0;
    for (int j = 0; j < m; ++j) s += Ainv[(long long)i * m + j] * r[j];
    u0[i] = s;
    u1[i] = s;
  }
}

// ---------------------------------------------------------------------------
// The coarse global levels in one workgroup.  Below a few thousand cells a
// level's operators are latency bound, and a launch per operator costs more
// than the work: k_fv_cycle runs every operator of levels 0..top (each of at
// most kCycMaxCells cells) in one 1024-thread workgroup on copies of the
// levels held in LDS, with a barrier between phases.  It performs either
//   mode 0: the FMG stages 0..top (Fig. 2): f of level top is restricted
//           down to level 0, u_0 = A^-1 f_0, then per level the trilinear
//           FMG step, S^cheb_fmg and one FAS V-cycle with rhs f_l, or
//   mode 1: one FAS V-cycle (Fig. 1) on level top, from its u and rhs.
// Each operator takes the arithmetic (and summation order) of its per-cell
// kernel above; Chebyshev steps alternate between two LDS copies of u.  The
// result, level top's u, goes to both of its global copies.
// ---------------------------------------------------------------------------
constexpr int kCycThreads = 1024;
constexpr int kCycMaxLevels = 8;
constexpr int kCycMaxCells = 1024;
constexpr int kCycArrays = 6;  // per level in LDS: u (two copies), rhs, t, r, f

struct CycleArgs {
  int top, mode;
  int n[kCycMaxLevels][3];
  double inv_h2[kCycMaxLevels];
  // Chebyshev step coefficients c_j = 1 / (d root_j) per level, j = 0..degree-1
  double cpre[kCycMaxLevels][8], cpost[kCycMaxLevels][8], cfmg[kCycMaxLevels][8];
  int dpre, dpost, dfmg;
  const double* Ainv;  // coarsest inverse (m0 x m0, global memory)
  int m0;
  const double* src;   // mode 0: f of level top; mode 1: rhs of level top
  const double* uin;   // mode 1: u of level top
  double* uout0;       // level top's result, both copies
  double* uout1;
  int o[kCycMaxLevels];  // LDS offset (doubles) of level l's kCycArrays arrays
};

__device__ inline int cyc_cells(const CycleArgs& A, int l) {
  return A.n[l][0] * A.n[l][1] * A.n[l][2];
}

// L v at cell (x, y, z) of a level stored plainly in LDS, odd reflection
// beyond the walls; the grouping of apply_L_direct
__device__ inline double cyc_L(const double* v, const int n[3], int x, int y, int z,
                               double inv_h2) {
  int ix[3], iy[3], iz[3];
  double sx[3], sy[3], sz[3];
  for (int k = 0; k < 3; ++k) {
    ix[k] = x + k - 1;
    iy[k] = y + k - 1;
    iz[k] = z + k - 1;
    sx[k] = mirror(n[0], ix[k]);
    sy[k] = mirror(n[1], iy[k]);
    sz[k] = mirror(n[2], iz[k]);
  }
  double P[3], Q[3];
  for (int c = 0; c < 3; ++c) {
    double a[3][3];
    for (int b = 0; b < 3; ++b)
      for (int e = 0; e < 3; ++e)
        a[b][e] = (sx[e] * sy[b] * sz[c]) * v[(iz[c] * n[1] + iy[b]) * n[0] + ix[e]];
    const double ctr = a[1][1];
    const double face = (a[1][0] + a[1][2]) + (a[0][1] + a[2][1]);
    const double corner = (a[0][0] + a[0][2]) + (a[2][0] + a[2][2]);
    P[c] = -4.0 * kW0 * ctr + (kW0 - 2.0 * kW1) * face + 2.0 * kW1 * corner;
    Q[c] = kW0 * kW0 * ctr + kW0 * kW1 * face + kW1 * kW1 * corner;
  }
  return (kW1 * (P[0] + P[2]) + kW0 * P[1] + (Q[0] + Q[2]) - 2.0 * Q[1]) * inv_h2;
}

__device__ inline void cyc_xyz(int i, const int n[3], int& x, int& y, int& z) {
  x = i % n[0];
  y = (i / n[0]) % n[1];
  z = i / (n[0] * n[1]);
}

// LDS arrays of level l: 0, 1 the copies of u, 2 rhs, 3 t, 4 r, 5 f
__device__ inline double* cyc_arr(double* sm, const CycleArgs& A, int l, int k) {
  return sm + A.o[l] + k * cyc_cells(A, l);
}

// deg Chebyshev steps on level l with right-hand side rhs; cur: bit l is the
// LDS copy holding u
__device__ void cyc_cheb(double* sm, const CycleArgs& A, int l, const double* rhs, int deg,
                         const double* coef, unsigned& cur) {
  const int cells = cyc_cells(A, l);
  for (int j = 0; j < deg; ++j) {
    const int c0 = (cur >> l) & 1;
    const double* u = cyc_arr(sm, A, l, c0);
    double* o = cyc_arr(sm, A, l, c0 ^ 1);
    for (int i = threadIdx.x; i < cells; i += kCycThreads) {
      int x, y, z;
      cyc_xyz(i, A.n[l], x, y, z);
      const double r = rhs[i] - cyc_L(u, A.n[l], x, y, z, A.inv_h2[l]);
      o[i] = u[i] - coef[j] * r;
    }
    cur ^= 1u << l;
    __syncthreads();
  }
}

// r = rhs - L u on level l, then, level l - 1: u = R u, r = R r (mean of the
// 8 children, in the order of mean8), rhs = r + L u (Eq. 4) and t = u
__device__ void cyc_descend(double* sm, const CycleArgs& A, int l, const double* rhs,
                            unsigned& cur) {
  const int cells = cyc_cells(A, l);
  const double* u = cyc_arr(sm, A, l, (cur >> l) & 1);
  double* r = cyc_arr(sm, A, l, 4);
  for (int i = threadIdx.x; i < cells; i += kCycThreads) {
    int x, y, z;
    cyc_xyz(i, A.n[l], x, y, z);
    r[i] = rhs[i] - cyc_L(u, A.n[l], x, y, z, A.inv_h2[l]);
  }
  __syncthreads();
  const int c = l - 1, cc = cyc_cells(A, c);
  cur &= ~(1u << c);
  double* uc = cyc_arr(sm, A, c, 0);
  double* rc = cyc_arr(sm, A, c, 4);
  const int* nf = A.n[l];
  for (int i = threadIdx.x; i < cc; i += kCycThreads) {
    int I, J, K;
    cyc_xyz(i, A.n[c], I, J, K);
    double su = 0.0, sr = 0.0;
    for (int cz = 0; cz < 2; ++cz)
      for (int b = 0; b < 2; ++b)
        for (int a = 0; a < 2; ++a) {
          const int f = ((2 * K + cz) * nf[1] + (2 * J + b)) * nf[0] + (2 * I + a);
          su += u[f];
          sr += r[f];
        }
    uc[i] = su / 8.0;
    rc[i] = sr / 8.0;
  }
  __syncthreads();
  double* rhc = cyc_arr(sm, A, c, 2);
  double* tc = cyc_arr(sm, A, c, 3);
  for (int i = threadIdx.x; i < cc; i += kCycThreads) {
    int x, y, z;
    cyc_xyz(i, A.n[c], x, y, z);
    tc[i] = uc[i];
    rhc[i] = rc[i] + cyc_L(uc, A.n[c], x, y, z, A.inv_h2[c]);
  }
  __syncthreads();
}

// level l's current u = P w (add = 0: the FMG step, w = level l - 1's u) or
// u += P (w - t) (add = 1: the correction); trilinear, odd reflection at the
// walls, the 8 terms in the order of k_fv_prolong
__device__ void cyc_prolong(double* sm, const CycleArgs& A, int l, int add, unsigned cur) {
  const int c = l - 1, cells = cyc_cells(A, l);
  const double* w = cyc_arr(sm, A, c, (cur >> c) & 1);
  const double* t = cyc_arr(sm, A, c, 3);
  double* u = cyc_arr(sm, A, l, (cur >> l) & 1);
  const int* nc = A.n[c];
  for (int i = threadIdx.x; i < cells; i += kCycThreads) {
    int fx, fy, fz;
    cyc_xyz(i, A.n[l], fx, fy, fz);
    const int p[3] = {fx >> 1, fy >> 1, fz >> 1};
    const int k[3] = {fx & 1, fy & 1, fz & 1};
    double s = 0.0;
    for (int cz = 0; cz < 2; ++cz)
      for (int cy = 0; cy < 2; ++cy)
        for (int cx = 0; cx < 2; ++cx) {
          const double wt = (cx ? 0.25 : 0.75) * (cy ? 0.25 : 0.75) * (cz ? 0.25 : 0.75);
          // the parent, or its neighbour toward the child
          int a = p[0] + (cx ? (k[0] ? 1 : -1) : 0);
          int b = p[1] + (cy ? (k[1] ? 1 : -1) : 0);
          int d = p[2] + (cz ? (k[2] ? 1 : -1) : 0);
          const double sg = mirror(nc[0], a) * mirror(nc[1], b) * mirror(nc[2], d);
          const int ci = (d * nc[1] + b) * nc[0] + a;
          const double cv = sg * (add ? w[ci] - t[ci] : w[ci]);
          s += wt * cv;
        }
    u[i] = add ? u[i] + s : s;
  }
  __syncthreads();
}

// u_0 = A^-1 rhs_0 (into both LDS copies of level 0)
__device__ void cyc_solve0(double* sm, const CycleArgs& A, const double* rhs, unsigned& cur) {
  double* u0 = cyc_arr(sm, A, 0, 0);
  double* u1 = cyc_arr(sm, A, 0, 1);
  for (int i = threadIdx.x; i < A.m0; i += kCycThreads) {
    double s = 0.0;
    for (int j = 0; j < A.m0; ++j) s += A.Ainv[(long long)i * A.m0 + j] * rhs[j];
    u0[i] = s;
    u1[i] = s;
  }
  cur &= ~1u;
  __syncthreads();
}

// FAS V-cycle from level top (right-hand side rt) down to the coarsest solve
// and back up (Fig. 1)
__device__ void cyc_vcycle(double* sm, const CycleArgs& A, int top, const double* rt,
                           unsigned& cur) {
  for (int l = top; l >= 1; --l) {
    const double* rhs = l == top ? rt : cyc_arr(sm, A, l, 2);
    cyc_cheb(sm, A, l, rhs, A.dpre, A.cpre[l], cur);
    cyc_descend(sm, A, l, rhs, cur);
  }
  cyc_solve0(sm, A, top == 0 ? rt : cyc_arr(sm, A, 0, 2), cur);
  for (int l = 1; l <= top; ++l) {
    const double* rhs = l == top ? rt : cyc_arr(sm, A, l, 2);
    cyc_prolong(sm, A, l, 1, cur);
    cyc_cheb(sm, A, l, rhs, A.dpost, A.cpost[l], cur);
  }
}

__global__ void __launch_bounds__(kCycThreads) k_fv_cycle(CycleArgs A) {
  extern __shared__ double cyc_sm[];
  double* sm = cyc_sm;
  const int top = A.top, ct = cyc_cells(A, top);
  unsigned cur = 0;  // bit l: the LDS copy of level l's u
  if (A.mode == 0) {
    double* f = cyc_arr(sm, A, top, 5);
    for (int i = threadIdx.x; i < ct; i += kCycThreads) f[i] = A.src[i];
    __syncthreads();
    for (int l = top; l >= 1; --l) {  // f_{l-1} = R f_l (mean8's order)
      const double* ff = cyc_arr(sm, A, l, 5);
      double* fc = cyc_arr(sm, A, l - 1, 5);
      const int* nf = A.n[l];
      for (int i = threadIdx.x; i < cyc_cells(A, l - 1); i += kCycThreads) {
        int I, J, K;
        cyc_xyz(i, A.n[l - 1], I, J, K);
        double sv = 0.0;
        for (int cz = 0; cz < 2; ++cz)
          for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 2; ++a)
              sv += ff[((2 * K + cz) * nf[1] + (2 * J + b)) * nf[0] + (2 * I + a)];
        fc[i] = sv / 8.0;
      }
      __syncthreads();
    }
    cyc_solve0(sm, A, cyc_arr(sm, A, 0, 5), cur);
    for (int l = 1; l <= top; ++l) {
      const double* fl = cyc_arr(sm, A, l, 5);
      cyc_prolong(sm, A, l, 0, cur);
      cyc_cheb(sm, A, l, fl, A.dfmg, A.cfmg[l], cur);
      cyc_vcycle(sm, A, l, fl, cur);
    }
  } else {
    double* rt = cyc_arr(sm, A, top, 2);
    double* u = cyc_arr(sm, A, top, 0);
    for (int i = threadIdx.x; i < ct; i += kCycThreads) {
      rt[i] = A.src[i];
      u[i] = A.uin[i];
    }
    __syncthreads();
    cyc_vcycle(sm, A, top, rt, cur);
  }
  const double* res = cyc_arr(sm, A, top, (cur >> top) & 1);
  for (int i = threadIdx.x; i < ct; i += kCycThreads) {
    A.uout0[i] = res[i];
    A.uout1[i] = res[i];
  }
}

// genuine cells of the finest segments into the caller's u (or a global
// level's copy into u)
__global__ void __launch_bounds__(kBlock) k_fv_gather(double* __restrict__ out,
                                                     const double* __restrict__ v, Geo G) {
  const int q = blockIdx.y;
  int vlo[3], vhi[3];
  seg_genuine(G, q, vlo, vhi);
  const int e[3] = {vhi[0] - vlo[0], vhi[1] - vlo[1], vhi[2] - vlo[2]};
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)e[0] * e[1] * e[2]) return;
  const int x = vlo[0] + (int)(t % e[0]), y = vlo[1] + (int)((t / e[0]) % e[1]),
            z = vlo[2] + (int)(t / ((long long)e[0] * e[1]));
  int clo[3], chi[3], slo[3];
  seg_region(G, q, clo, chi, slo);
  out[((long long)z * G.n[1] + y) * G.n[0] + x] = v[sidx(G, q, slo, x, y, z)];
}

// ---------------------------------------------------------------------------
// host: plan and schedule
// ---------------------------------------------------------------------------

struct Level {
  Geo G;
  double h;
  double* u[2] = {nullptr, nullptr};  // two copies
  int cur = 0;                        // copy holding the current iterate
  double* rhs = nullptr;              // segment / coarse right-hand side
  double* t = nullptr;                // copy of the restricted u
  double* r = nullptr;                // residual, then restricted residual
  double* f = nullptr;                // FMG right-hand side (global array)
};

}  // namespace fv

struct fv27_plan {
  fv27_params p;
  std::vector<int32_t> J;
  int device = 0;
  int L = 0, K = 0, T = 0;
  std::vector<fv::Level> lv;
  std::vector<void*> allocs;
  double* Ainv = nullptr;
  int m0 = 0;
  int64_t bytes = 0;
  int Lc = -1;  // levels 0..Lc run in k_fv_cycle (-1: none)
  long long march_slots = 256 * 8;   // march workgroups resident at once (CUs x occupancy)
  long long march2_slots = 256 * 4;  // ... of the two-step march
  // schedule model of the last walk
  int64_t launches = 0;
  double model_bytes = 0.0;
};

namespace fv {

static const char* check(const fv27_params* p) {
  if (!p) return "params is NULL";
  if (!(p->h > 0.0) || !std::isfinite(p->h)) return "h must be positive and finite";
  if (p->levels < 1 || p->levels > 24) return "levels must be in [1, 24]";
  long long m = 1;
  for (int d = 0; d < 3; ++d) {
    if (p->n[d] < 1) return "every extent must be >= 1";
    if ((p->n[d] >> (p->levels - 1)) << (p->levels - 1) != p->n[d])
      return "every extent must be divisible by 2^(levels-1)";
    m *= p->n[d] >> (p->levels - 1);
  }
  if (m > kMaxCoarse) return "the coarsest level must have at most 512 cells";
  if ((long long)p->n[0] * p->n[1] * p->n[2] > (1ll << 33)) return "grid too large";
  if (p->cheb_pre < 0 || p->cheb_pre > 8 || p->cheb_post < 0 || p->cheb_post > 8 ||
      p->cheb_fmg < 0 || p->cheb_fmg > 8)
    return "Chebyshev degrees must be in [0, 8]";
  const int K = p->sr_levels;
  if (K < 0 || K > p->levels - 1) return "sr_levels must be in [0, levels-1]";
  if (K == 0) return nullptr;
  if (!p->buffer_schedule) return "buffer_schedule is NULL";
  for (int d = 0; d < 3; ++d) {
    if (p->segments[d] < 1) return "segments must be >= 1";
    if (p->n[d] % ((long long)p->segments[d] << K) != 0)
      return "every extent must be divisible by segments << sr_levels";
  }
  if (p->n[0] / p->segments[0] != p->n[1] / p->segments[1] ||
      p->n[0] / p->segments[0] != p->n[2] / p->segments[2])
    return "segments must be cubic (n[d] / segments[d] equal for all d)";
  for (int i = 0; i < K; ++i) {
    const int j = p->buffer_schedule[i];
    if (j < 0 || (j & 1)) return "buffer widths must be even and >= 0";
    if (j > (1 << 20)) return "buffer width too large";
    if (i + 1 < K && 2 * p->buffer_schedule[i + 1] < j)
      return "each buffer width must be at least half the next finer one";
  }
  return nullptr;
}

// exact inverse of the coarsest operator (Gauss-Jordan with partial pivoting)
static std::vector<double> coarse_inverse(const int n[3], double h) {
  const int m = n[0] * n[1] * n[2];
  std::vector<double> A((size_t)m * m, 0.0), I((size_t)m * m, 0.0);
  auto refl = [](int nn, int& i) -> double {
    if (i < 0) {
      i = -1 - i;
      return -1.0;
    }
    if (i >= nn) {
      i = 2 * nn - 1 - i;
      return -1.0;
    }
    return 1.0;
  };
  const double w[3] = {kW1, kW0, kW1};
  const double d2[3] = {1.0, -2.0, 1.0};
  for (int z = 0; z < n[2]; ++z)
    for (int y = 0; y < n[1]; ++y)
      for (int x = 0; x < n[0]; ++x) {
        const int row = (z * n[1] + y) * n[0] + x;
        for (int c = 0; c < 3; ++c)
          for (int b = 0; b < 3; ++b)
            for (int a = 0; a < 3; ++a) {
              const double coef =
                  (d2[a] * w[b] * w[c] + w[a] * d2[b] * w[c] + w[a] * w[b] * d2[c]) / (h * h);
              int i = x + a - 1, j = y + b - 1, k = z + c - 1;
              const double s = refl(n[0], i) * refl(n[1], j) * refl(n[2], k);
              A[(size_t)row * m + (k * n[1] + j) * n[0] + i] += s * coef;
            }
      }
  for (int i = 0; i < m; ++i) I[(size_t)i * m + i] = 1.0;
  for (int c = 0; c < m; ++c) {
    int best = c;
    for (int r = c + 1; r < m; ++r)
      if (std::fabs(A[(size_t)r * m + c]) > std::fabs(A[(size_t)best * m + c])) best = r;
    if (best != c)
      for (int t = 0; t < m; ++t) {
        std::swap(A[(size_t)c * m + t], A[(size_t)best * m + t]);
        std::swap(I[(size_t)c * m + t], I[(size_t)best * m + t]);
      }
    const double piv = A[(size_t)c * m + c];
    for (int t = 0; t < m; ++t) {
      A[(size_t)c * m + t] /= piv;
      I[(size_t)c * m + t] /= piv;
    }
    for (int r = 0; r < m; ++r) {
      if (r == c) continue;
      const double l = A[(size_t)r * m + c];
      if (l == 0.0) continue;
      for (int t = 0; t < m; ++t) {
        A[(size_t)r * m + t] -= l * A[(size_t)c * m + t];
        I[(size_t)r * m + t] -= l * I[(size_t)c * m + t];
      }
    }
  }
  return I;
}

static double cheb_root(int j, int k) {
  const double pi = 3.14159265358979323846;
  const double a = 48.0 / 121.0, b = 200.0 / 121.0;
  return 0.5 * (a + b) + 0.5 * (b - a) * std::cos((2.0 * j - 1.0) * pi / (2.0 * k));
}

static unsigned blocks_for(long long cells) { return (unsigned)((cells + kBlock - 1) / kBlock); }

// coarse parents of the fine cells a prolongation writes, at most, per segment
static long long parents(const Geo& G) {
  long long c = 1;
  for (int d = 0; d < 3; ++d) c *= G.sr ? ((G.m[d] + 1) >> 1) + 1 : (G.n[d] + 1) >> 1;
  return c;
}

// One solve's launches (or, with dry, only their count and bytes).
struct Exec {
  fv27_plan* P;
  hipStream_t s;
  bool dry;

  void count(double bytes) {
    P->launches += 1;
    P->model_bytes += bytes;
  }
  void launched() {
    if (!dry) hipcheck(hipGetLastError(), "kernel launch");
  }

  // cells of the compute regions of a level (all segments)
  static double c_cells(const Geo& G) {
    double s = 0.0;
    for (int q = 0; q < nseg(G); ++q) {
      int lo[3], hi[3], sl[3];
      seg_region(G, q, lo, hi, sl);
      s += (double)(hi[0] - lo[0]) * (hi[1] - lo[1]) * (hi[2] - lo[2]);
    }
    return s;
  }
  static double storage_cells(const Geo& G) {
    double s = 0.0;
    for (int q = 0; q < nseg(G); ++q) {
      int lo[3], hi[3], sl[3];
      seg_region(G, q, lo, hi, sl);
      double c = 1.0;
      for (int d = 0; d < 3; ++d) {
        int a = G.sr ? std::max(0, lo[d] - 1) : 0, b = G.sr ? std::min(G.n[d], hi[d] + 1) : G.n[d];
        c *= (double)(b - a);
      }
      s += c;
    }
    return s;
  }

  // one march pass over level l: mode 0 Chebyshev step (cur -> other), mode 1
  // residual into lv.r
  void march(int l, const double* rhs, bool rhs_global, int mode, double c,
             double* fin_u = nullptr) {
    Level& V = P->lv[l];
    const Geo& G = V.G;
    MarchArgs A{};
    A.G = G;
    A.fin = fin_u;
    A.u = V.u[V.cur];
    A.out = mode ? V.r : V.u[V.cur ^ 1];
    A.rhs = rhs;
    A.rhs_global = rhs_global ? 1 : 0;
    A.mode = mode;
    A.c = c;
    A.inv_h2 = 1.0 / (V.h * V.h);
    int ext[3];
    if (G.sr) {
      for (int d = 0; d < 3; ++d) ext[d] = std::min(G.n[d], G.g + 2 * G.J);
    } else {
      for (int d = 0; d < 3; ++d) ext[d] = G.n[d];
    }
    A.tiles_x = (ext[0] + kTX - 1) / kTX;
    const int tiles_y = (ext[1] + kTY - 1) / kTY;
    A.zchunk = zchunk_for(ext[2], (long long)A.tiles_x * tiles_y * nseg(G), P->march_slots, 2);
    const int chunks = (ext[2] + A.zchunk - 1) / A.zchunk;
    count(c_cells(G) * 24.0 + (fin_u ? 8.0 * G.n[0] * G.n[1] * G.n[2] : 0.0));
    if (dry) {
      if (mode == 0) V.cur ^= 1;
      return;
    }
    hipLaunchKernelGGL(k_fv_march, dim3((unsigned)(A.tiles_x * tiles_y), (unsigned)chunks,
                                        (unsigned)nseg(G)),
                       dim3(kThreads), 0, s, A);
    launched();
    if (mode == 0) V.cur ^= 1;
  }

  // z chunks of a march over `ext` planes with `cols` tile columns: the fewest
  // rounds of resident workgroups times the planes a chunk marches (its own
  // plus `halo`), the last round counted whole; ties to fewer, longer chunks
  static int zchunk_for(int ext, long long cols, long long slots, int halo) {
    long long bestc = -1;
    int best = ext;
    for (int nz = 1; nz <= ext; ++nz) {
      const int zc = (ext + nz - 1) / nz;
      const long long blocks = cols * ((ext + zc - 1) / zc);
      const long long c = ((blocks + slots - 1) / slots) * (zc + halo);
      if (bestc < 0 || c < bestc) {
        bestc = c;
        best = zc;
      }
    }
    return best;
  }

  // two Chebyshev steps (coefficients c and c2) in one temporally blocked
  // pass over level l (cur -> other)
  void march2(int l, const double* rhs, bool rhs_global, double c, double c2,
              double* fin_u = nullptr) {
    Level& V = P->lv[l];
    const Geo& G = V.G;
    MarchArgs A{};
    A.G = G;
    A.fin = fin_u;
    A.u = V.u[V.cur];
    A.out = V.u[V.cur ^ 1];
    A.rhs = rhs;
    A.rhs_global = rhs_global ? 1 : 0;
    A.mode = 0;
    A.c = c;
    A.inv_h2 = 1.0 / (V.h * V.h);
    int ext[3];
    for (int d = 0; d < 3; ++d) ext[d] = G.sr ? std::min(G.n[d], G.g + 2 * G.J) : G.n[d];
    A.tiles_x = (ext[0] + kTX - 1) / kTX;
    const int tiles_y = (ext[1] + kTY - 1) / kTY;
    A.zchunk = zchunk_for(ext[2], (long long)A.tiles_x * tiles_y * nseg(G), P->march2_slots, 4);
    const int chunks = (ext[2] + A.zchunk - 1) / A.zchunk;
    count(c_cells(G) * 24.0 + (fin_u ? 8.0 * G.n[0] * G.n[1] * G.n[2] : 0.0));
    V.cur ^= 1;
    if (dry) return;
    hipLaunchKernelGGL(k_fv_march2, dim3((unsigned)(A.tiles_x * tiles_y), (unsigned)chunks,
                                         (unsigned)nseg(G)),
                       dim3(kThreads2), 0, s, A, c2);
    launched();
  }

  // the caller's u while the solve's last smoothing runs: its last step
  // writes the genuine cells there too, and no gather is needed
  double* fin = nullptr;
  bool fin_done = false;
  bool fused2 = true;  // two Chebyshev steps per pass

  void cheb(int l, const double* rhs, bool rhs_global, int degree, bool last = false) {
    Level& V = P->lv[l];
    const double d = (121.0 / 24.0) / (V.h * V.h);
    // steps in pairs, each pair one temporally blocked pass
    // (the two-step pass reads two cells beyond a wall: every extent >= 2).
    // Segment levels, and global levels above 2M cells, keep one step per
    // pass: the two-step pass holds two workgroups of 512 threads per CU (106
    // VGPRs), too few to hide its per-plane latency, and measured slower there
    // (512 x 256 x 256: 576 us against two 260 us steps; 256 x 128 x 128: 68
    // against two 31 us; every segment level of the model problem; at
    // 128 x 64 x 64 the pair is faster, 17 against two 11 us).
    const long long cells = (long long)V.G.n[0] * V.G.n[1] * V.G.n[2];
    const bool two = fused2 && !V.G.sr && cells <= (2ll << 20) && V.G.n[0] >= 2 &&
                     V.G.n[1] >= 2 && V.G.n[2] >= 2;
    for (int j = 1; j <= degree;) {
      double* fo = last && (j == degree || (two && j + 1 == degree)) ? fin : nullptr;
      if (two && j + 1 <= degree) {
        march2(l, rhs, rhs_global, 1.0 / (d * cheb_root(j, degree)),
               1.0 / (d * cheb_root(j + 1, degree)), fo);
        j += 2;
      } else {
        march(l, rhs, rhs_global, 0, 1.0 / (d * cheb_root(j, degree)), fo);
        j += 1;
      }
    }
    if (last && degree > 0 && fin) fin_done = true;
  }

  // restriction of u (and the residual) from level l into level l-1
  void restrict_level(int l, int target) {
    Level& F = P->lv[l];
    Level& C = P->lv[l - 1];
    RestrictArgs A{};
    A.F = F.G;
    A.C = C.G;
    A.fu = F.u[F.cur];
    A.fr = F.r;
    A.cu = C.u[C.cur];
    A.cr = C.r;
    A.target = target;
    int ex[3];
    if (target == 0) {
      for (int d = 0; d < 3; ++d) ex[d] = C.G.n[d];
    } else if (target == 1) {
      for (int d = 0; d < 3; ++d) ex[d] = std::min(F.G.n[d], F.G.g + 2 * F.G.J) / 2;
    } else {
      for (int d = 0; d < 3; ++d) ex[d] = F.G.g / 2;
    }
    for (int d = 0; d < 3; ++d) A.ex[d] = ex[d];
    const long long cells = (long long)ex[0] * ex[1] * ex[2];
    count((double)cells * nseg(F.G) * (16.0 * 8 + 16.0));
    if (dry) return;
    hipLaunchKernelGGL(k_fv_restrict, dim3(blocks_for(cells), (unsigned)nseg(F.G)), dim3(kBlock), 0,
                       s, A);
    launched();
  }

  void fas(int l) {  // coarse level l - 1 of fine level l
    Level& F = P->lv[l];
    Level& C = P->lv[l - 1];
    FasArgs A{};
    A.C = C.G;
    A.F = F.G;
    A.u = C.u[C.cur];
    A.rr = C.r;
    A.rhs = C.rhs;
    A.t = C.t;
    A.inv_h2 = 1.0 / (C.h * C.h);
    count(storage_cells(C.G) * 16.0 + c_cells(C.G) * 16.0);
    if (dry) return;
    hipLaunchKernelGGL(k_fv_fas, dim3(blocks_for(C.G.box), (unsigned)nseg(C.G)), dim3(kBlock), 0, s,
                       A);
    launched();
  }

  // FMG step (add = 0, source u of level l-1) or correction (add = 1)
  void prolong(int l, int add) {
    Level& F = P->lv[l];
    Level& C = P->lv[l - 1];
    ProlongArgs A{};
    A.F = F.G;
    A.C = C.G;
    A.csrc_seg = C.G.sr;
    A.w = C.u[C.cur];
    A.t = add ? C.t : nullptr;
    A.u0 = F.u[F.cur];
    A.u1 = F.u[F.cur ^ 1];
    A.add = add;
    const double fc = storage_cells(F.G), gh = fc - c_cells(F.G);
    count(fc * (add ? 16.0 : 8.0) + gh * 8.0 + storage_cells(C.G) * (add ? 16.0 : 8.0));
    if (dry) return;
    hipLaunchKernelGGL(k_fv_prolong, dim3(blocks_for(parents(F.G)), (unsigned)nseg(F.G)),
                       dim3(kBlock), 0, s, A);
    launched();
  }

  void coarse_solve(const double* rhs) {
    Level& V = P->lv[0];
    count(P->m0 * 24.0 + (double)P->m0 * P->m0 * 8.0);
    if (dry) return;
    hipLaunchKernelGGL(k_fv_coarse, dim3(1), dim3(kBlock), 0, s, (const double*)P->Ainv, P->m0, rhs,
                       V.u[0], V.u[1]);
    launched();
  }

  // levels 0..Lc in one workgroup: mode 0, the FMG stages 0..Lc (src = f of
  // level Lc); mode 1, the V-cycle on level Lc (src = its right-hand side)
  void cycle(int mode, const double* src) {
    const int top = P->Lc;
    Level& V = P->lv[top];
    CycleArgs A{};
    A.top = top;
    A.mode = mode;
    int off = 0;
    for (int l = 0; l <= top; ++l) {
      const Level& W = P->lv[l];
      for (int d = 0; d < 3; ++d) A.n[l][d] = W.G.n[d];
      A.inv_h2[l] = 1.0 / (W.h * W.h);
      const double d = (121.0 / 24.0) / (W.h * W.h);
      for (int j = 1; j <= P->p.cheb_pre; ++j) A.cpre[l][j - 1] = 1.0 / (d * cheb_root(j, P->p.cheb_pre));
      for (int j = 1; j <= P->p.cheb_post; ++j)
        A.cpost[l][j - 1] = 1.0 / (d * cheb_root(j, P->p.cheb_post));
      for (int j = 1; j <= P->p.cheb_fmg; ++j) A.cfmg[l][j - 1] = 1.0 / (d * cheb_root(j, P->p.cheb_fmg));
      A.o[l] = off;
      off += kCycArrays * W.G.n[0] * W.G.n[1] * W.G.n[2];
    }
    A.dpre = P->p.cheb_pre;
    A.dpost = P->p.cheb_post;
    A.dfmg = P->p.cheb_fmg;
    A.Ainv = P->Ainv;
    A.m0 = P->m0;
    A.src = src;
    A.uin = V.u[V.cur];
    A.uout0 = V.u[0];
    A.uout1 = V.u[1];
    const double ct = (double)V.G.n[0] * V.G.n[1] * V.G.n[2];
    count(ct * (mode ? 32.0 : 24.0) + (double)P->m0 * P->m0 * 8.0);
    if (dry) return;
    hipLaunchKernelGGL(k_fv_cycle, dim3(1), dim3(kCycThreads), (size_t)off * sizeof(double), s, A);
    launched();
  }

  // FAS V-cycle on global level l (Fig. 1)
  void vcycle_global(int l, const double* rhs) {
    Level& V = P->lv[l];
    if (l == P->Lc) {
      cycle(1, rhs);
      return;
    }
    if (l == 0) {
      coarse_solve(rhs);
      return;
    }
    cheb(l, rhs, true, P->p.cheb_pre);
    march(l, rhs, true, 1, 0.0);
    restrict_level(l, 0);
    fas(l);
    vcycle_global(l - 1, P->lv[l - 1].rhs);
    prolong(l, 1);
    cheb(l, rhs, true, P->p.cheb_post, l == P->L - 1);
    (void)V;
  }

  // FAS V-cycle with segmental refinement on SR level l (Fig. 6); top is the
  // level of the current FMG stage, whose right-hand side is the global f
  void vcycle_sr(int l, int top) {
    Level& V = P->lv[l];
    const bool atop = l == top;
    const double* rhs = atop ? V.f : V.rhs;
    cheb(l, rhs, atop, P->p.cheb_pre);
    march(l, rhs, atop, 1, 0.0);
    if (l - 1 > P->T) {
      restrict_level(l, 1);
      fas(l);
      vcycle_sr(l - 1, top);
    } else {
      restrict_level(l, 2);
      fas(l);
      vcycle_global(l - 1, P->lv[l - 1].rhs);
    }
    prolong(l, 1);
    cheb(l, rhs, atop, P->p.cheb_post, l == P->L - 1);
  }

  void f_hierarchy(const double* f) {
    P->lv[P->L - 1].f = const_cast<double*>(f);
    // (k_fv_cycle restricts f below level Lc itself)
    for (int l = P->L - 1; l > std::max(P->Lc, 0); --l) {
      Level& F = P->lv[l];
      Level& C = P->lv[l - 1];
      RestrictArgs A{};
      A.F = global_geo(F.G.n);
      A.C = global_geo(C.G.n);
      A.fu = F.f;
      A.fr = nullptr;
      A.cu = C.f;
      A.cr = nullptr;
      A.target = 0;
      for (int d = 0; d < 3; ++d) A.ex[d] = C.G.n[d];
      const long long cells = (long long)A.ex[0] * A.ex[1] * A.ex[2];
      count((double)cells * 72.0);
      if (dry) continue;
      hipLaunchKernelGGL(k_fv_restrict, dim3(blocks_for(cells), 1), dim3(kBlock), 0, s, A);
      launched();
    }
  }

  void solve(const double* f, double* u) {
    const int L = P->L;
    for (auto& V : P->lv) V.cur = 0;
    fin = dry ? (double*)(uintptr_t)1 : u;  // (a dry walk only counts)
    fin_done = false;
    f_hierarchy(f);
    // global FMG stages 0..T (Fig. 2); stages 0..Lc in one launch
    int l0 = 1;
    if (P->Lc >= 1) {
      cycle(0, P->lv[P->Lc].f);
      l0 = P->Lc + 1;
    } else {
      coarse_solve(P->lv[0].f);
    }
    for (int l = l0; l <= P->T; ++l) {
      prolong(l, 0);
      cheb(l, P->lv[l].f, true, P->p.cheb_fmg);
      vcycle_global(l, P->lv[l].f);
    }
    // segment stages T+1..L-1 (Fig. 5)
    for (int top = P->T + 1; top < L; ++top) {
      prolong(top, 0);
      cheb(top, P->lv[top].f, true, P->p.cheb_fmg);
      vcycle_sr(top, top);
    }
    // output: the genuine cells of the finest level, unless its last
    // smoothing step wrote them (no post-smoothing, or a one-level solve)
    if (fin_done) return;
    Level& V = P->lv[L - 1];
    const Geo& G = V.G;
    const long long cells = G.sr ? (long long)G.g * G.g * G.g : G.box;
    count((double)G.n[0] * G.n[1] * G.n[2] * 16.0);
    if (dry) return;
    Geo Gg = G;
    if (!G.sr) {  // one global segment: genuine = the whole level
      Gg.S[0] = Gg.S[1] = Gg.S[2] = 1;
    }
    hipLaunchKernelGGL(k_fv_gather, dim3(blocks_for(cells), (unsigned)nseg(G)), dim3(kBlock), 0, s, u,
                       (const double*)V.u[V.cur], Gg);
    launched();
  }
};

static void release(fv27_plan* P) {
  for (void* p : P->allocs) (void)hipFree(p);
  P->allocs.clear();
  delete P;
}

static double* dalloc(fv27_plan* P, size_t bytes) {
  void* p = nullptr;
  if (bytes == 0) bytes = 8;
  if (hipMalloc(&p, bytes) != hipSuccess) throw hip_error{"hipMalloc failed"};
  P->allocs.push_back(p);
  P->bytes += (int64_t)bytes;
  hipcheck(hipMemset(p, 0, bytes), "hipMemset");
  return (double*)p;
}

static void walk_model(fv27_plan* P) {
  P->launches = 0;
  P->model_bytes = 0.0;
  Exec E{P, nullptr, true};
  E.solve(nullptr, nullptr);
}

}  // namespace fv

extern "C" {

int32_t fv27_check_params(const fv27_params* p) {
  const char* m = fv::check(p);
  return m ? fv::fail(FMG_EINVAL, m) : FMG_OK;
}

int32_t fv27_plan_create(const fv27_params* p, int32_t device, fv27_plan** out) {
  if (!out) return fv::fail(FMG_EINVAL, "out is NULL");
  *out = nullptr;
  if (const char* m = fv::check(p)) return fv::fail(FMG_EINVAL, m);
  fv27_plan* P = new fv27_plan();
  P->p = *p;
  if (p->sr_levels > 0) P->J.assign(p->buffer_schedule, p->buffer_schedule + p->sr_levels);
  P->p.buffer_schedule = P->J.empty() ? nullptr : P->J.data();
  P->device = device;
  P->L = p->levels;
  P->K = p->sr_levels;
  P->T = P->L - 1 - P->K;
  // the coarse-cycle kernel takes the global levels of at most kCycMaxCells
  // cells (its LDS then stays under 64 KiB), if there are at least two
  P->Lc = -1;
  for (int l = 0; l <= P->T && l < fv::kCycMaxLevels; ++l) {
    const int sh = P->L - 1 - l;
    if ((long long)(p->n[0] >> sh) * (p->n[1] >> sh) * (p->n[2] >> sh) > fv::kCycMaxCells) break;
    P->Lc = l;
  }
  if (P->Lc < 1) P->Lc = -1;
  try {
    fv::hipcheck(hipSetDevice(device), "hipSetDevice");
    P->lv.resize(P->L);
    for (int l = 0; l < P->L; ++l) {
      fv::Level& V = P->lv[l];
      const int sh = P->L - 1 - l;
      int n[3] = {p->n[0] >> sh, p->n[1] >> sh, p->n[2] >> sh};
      V.h = p->h * (double)(1ll << sh);
      V.G = (l > P->T) ? fv::seg_geo(n, p->segments, P->J[P->L - 1 - l]) : fv::global_geo(n);
      const size_t cells = (size_t)V.G.box * fv::nseg(V.G);
      V.u[0] = fv::dalloc(P, cells * sizeof(double));
      V.u[1] = fv::dalloc(P, cells * sizeof(double));
      V.rhs = fv::dalloc(P, cells * sizeof(double));
      V.t = fv::dalloc(P, cells * sizeof(double));
      V.r = fv::dalloc(P, cells * sizeof(double));
      if (l < P->L - 1) V.f = fv::dalloc(P, (size_t)n[0] * n[1] * n[2] * sizeof(double));
    }
    int ncu = 0, occ = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess &&
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fv::k_fv_march, fv::kThreads, 0) ==
            hipSuccess &&
        ncu > 0 && occ > 0)
      P->march_slots = (long long)ncu * occ;
    else
      (void)hipGetLastError();
    occ = 0;
    if (ncu > 0 &&
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fv::k_fv_march2, fv::kThreads2, 0) ==
            hipSuccess &&
        occ > 0)
      P->march2_slots = (long long)ncu * occ;
    else
      (void)hipGetLastError();
    int n0[3] = {p->n[0] >> (P->L - 1), p->n[1] >> (P->L - 1), p->n[2] >> (P->L - 1)};
    P->m0 = n0[0] * n0[1] * n0[2];
    std::vector<double> inv = fv::coarse_inverse(n0, P->lv[0].h);
    P->Ainv = fv::dalloc(P, inv.size() * sizeof(double));
    fv::hipcheck(hipMemcpy(P->Ainv, inv.data(), inv.size() * sizeof(double), hipMemcpyHostToDevice),
                 "hipMemcpy");
    fv::walk_model(P);
  } catch (const fv::hip_error& e) {
    fv::release(P);
    return fv::fail(e.what.find("hipMalloc") != std::string::npos ? FMG_ENOMEM : FMG_EHIP, e.what);
  }
  *out = P;
  return FMG_OK;
}

int32_t fv27_plan_execute(fv27_plan* P, const double* f, double* u, void* stream) {
  if (!P) return fv::fail(FMG_EINVAL, "plan is NULL");
  if (!f || !u) return fv::fail(FMG_EINVAL, "f or u is NULL");
  const size_t bytes = sizeof(double) * (size_t)P->p.n[0] * P->p.n[1] * P->p.n[2];
  const char* fa = (const char*)f;
  const char* ua = (const char*)u;
  if (fa < ua + bytes && ua < fa + bytes) return fv::fail(FMG_EINVAL, "f and u overlap");
  try {
    fv::hipcheck(hipSetDevice(P->device), "hipSetDevice");
    fv::Exec E{P, (hipStream_t)stream, false};
    const int64_t l0 = P->launches;
    const double b0 = P->model_bytes;
    E.solve(f, u);
    P->launches = l0;
    P->model_bytes = b0;
  } catch (const fv::hip_error& e) {
    return fv::fail(FMG_EHIP, e.what);
  }
  return FMG_OK;
}

int32_t fv27_plan_destroy(fv27_plan* P) {
  if (!P) return FMG_OK;
  (void)hipSetDevice(P->device);
  (void)hipDeviceSynchronize();
  fv::release(P);
  return FMG_OK;
}

int64_t fv27_plan_workspace_bytes(const fv27_plan* P) { return P ? P->bytes : 0; }

int32_t fv27_plan_model(const fv27_plan* P, int64_t* launches, double* bytes) {
  if (!P) return fv::fail(FMG_EINVAL, "plan is NULL");
  if (launches) *launches = P->launches;
  if (bytes) *bytes = P->model_bytes;
  return FMG_OK;
}

static fv::MarchArgs whole_box_march(const int32_t* n, double h) {
  fv::MarchArgs A{};
  int nn[3] = {n[0], n[1], n[2]};
  A.G = fv::global_geo(nn);
  A.inv_h2 = 1.0 / (h * h);
  A.rhs = nullptr;
  A.rhs_global = 1;
  A.c = 0.0;
  A.tiles_x = (n[0] + fv::kTX - 1) / fv::kTX;
  A.zchunk = 8;
  A.fin = nullptr;  // single operators deliver nothing beyond `out`
  return A;
}

static hipError_t launch_march(const fv::MarchArgs& A, const int32_t* n, hipStream_t s) {
  const int tiles_y = (n[1] + fv::kTY - 1) / fv::kTY;
  const int chunks = (n[2] + A.zchunk - 1) / A.zchunk;
  hipLaunchKernelGGL(fv::k_fv_march, dim3((unsigned)(A.tiles_x * tiles_y), (unsigned)chunks, 1),
                     dim3(fv::kThreads), 0, s, A);
  return hipGetLastError();
}

static bool bad_box(const int32_t* n, double h) {
  return !n || n[0] < 1 || n[1] < 1 || n[2] < 1 || !(h > 0.0) ||
         (long long)n[0] * n[1] * n[2] > (1ll << 31);
}

int32_t fv27_op_apply(const double* u, const int32_t* n, double h, double* out, void* stream) {
  if (!u || !out || bad_box(n, h) || u == out) return fv::fail(FMG_EINVAL, "bad arguments");
  fv::MarchArgs A = whole_box_march(n, h);
  A.u = u;
  A.out = out;
  A.mode = 2;
  hipError_t e = launch_march(A, n, (hipStream_t)stream);
  return e == hipSuccess ? FMG_OK : fv::fail(FMG_EHIP, hipGetErrorString(e));
}

int32_t fv27_op_cheb(double* u, const double* rhs, const int32_t* n, double h, int32_t degree,
                     void* stream) {
  if (!u || !rhs || bad_box(n, h) || degree < 0 || degree > 8 || (const double*)u == rhs)
    return fv::fail(FMG_EINVAL, "bad arguments");
  const size_t bytes = sizeof(double) * (size_t)n[0] * n[1] * n[2];
  hipStream_t s = (hipStream_t)stream;
  double* tmp = nullptr;
  if (hipMalloc(&tmp, bytes) != hipSuccess) return fv::fail(FMG_ENOMEM, "hipMalloc failed");
  fv::MarchArgs A = whole_box_march(n, h);
  A.rhs = rhs;
  A.mode = 0;
  const double d = (121.0 / 24.0) / (h * h);
  double* cur = u;
  double* oth = tmp;
  hipError_t e = hipSuccess;
  // steps in pairs through the two-step pass (every extent >= 2), as the solver does on
  // global levels of up to 2M cells
  const bool two = n[0] >= 2 && n[1] >= 2 && n[2] >= 2;
  for (int j = 1; j <= degree && e == hipSuccess;) {
    A.u = cur;
    A.out = oth;
    A.c = 1.0 / (d * fv::cheb_root(j, degree));
    if (two && j + 1 <= degree) {
      const double c2 = 1.0 / (d * fv::cheb_root(j + 1, degree));
      const int tiles_y = (n[1] + fv::kTY - 1) / fv::kTY;
      const int chunks = (n[2] + A.zchunk - 1) / A.zchunk;
      hipLaunchKernelGGL(fv::k_fv_march2, dim3((unsigned)(A.tiles_x * tiles_y), (unsigned)chunks, 1),
                         dim3(fv::kThreads2), 0, s, A, c2);
      e = hipGetLastError();
      j += 2;
    } else {
      e = launch_march(A, n, s);
      j += 1;
    }
    std::swap(cur, oth);
  }
  if (e == hipSuccess && cur != u) e = hipMemcpyAsync(u, cur, bytes, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(tmp);
  return e == hipSuccess ? FMG_OK : fv::fail(FMG_EHIP, hipGetErrorString(e));
}

int32_t fv27_op_prolong(const double* coarse, const int32_t* n, double* fine, void* stream) {
  if (!coarse || !fine || bad_box(n, 1.0) || (long long)n[0] * n[1] * n[2] > (1ll << 27))
    return fv::fail(FMG_EINVAL, "bad arguments");
  int nc[3] = {n[0], n[1], n[2]}, nf[3] = {2 * n[0], 2 * n[1], 2 * n[2]};
  fv::ProlongArgs A{};
  A.F = fv::global_geo(nf);
  A.C = fv::global_geo(nc);
  A.csrc_seg = 0;
  A.w = coarse;
  A.t = nullptr;
  A.u0 = fine;
  A.u1 = fine;
  A.add = 0;
  hipLaunchKernelGGL(fv::k_fv_prolong, dim3(fv::blocks_for(fv::parents(A.F)), 1),
                     dim3(fv::kBlock), 0, (hipStream_t)stream, A);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? FMG_OK : fv::fail(FMG_EHIP, hipGetErrorString(e));
}

const char* fv27_last_error(void) { return fv::g_err.c_str(); }

}  // extern "C"
