// grid.hpp -- level and segment geometry shared by the host schedule and the
// device kernels.
//
// Every level of the hierarchy is stored as one or more boxes.  A global level
// (Sec. 3.3 of the paper, the conventional solver up to the transition level)
// is a single unpadded n^3 box.  A segmental-refinement level (Sec. 4) holds
// S^3 boxes, one per segment p = (px,py,pz): the compute region
//   C = [max(0, p g - J), min(n, (p+1) g + J))   per dimension, g = n / S,
// grown by one ghost layer (ghost cells inside the domain are the frozen GSR
// cells, those outside are boundary ghosts and are never touched).  All boxes
// of a level share the edge m = min(n, g + 2J) + 2 so segment q starts at
// element q * m^3; clipped boxes leave their tail unused.
#pragma once
#include <hip/hip_runtime.h>

namespace fmg {

struct Geo {
  int n;          // level edge: the domain is cells [0, n)^3 of this level
  int S;          // segments per dimension (1 for a global level)
  int g;          // genuine edge n / S
  int J;          // buffer width
  int m;          // storage edge per dimension
  int ghost;      // 1: storage starts one cell before C; 0: unpadded global
  long long sstride;  // elements from one segment's box to the next
};

struct Box {
  int a[3];   // compute region start (global level indices)
  int b[3];   // compute region end (exclusive)
  int o[3];   // global index of storage element (0,0,0)
  long long base;
};

// floor(a / b) for 0 <= a < 2^22 and 1 <= b < 2^11.  The product with the
// hardware reciprocal (relative error below 2^-22) lies within one of a / b,
// so its truncation is the quotient or one off, which one test corrects.
// (A 32-bit integer division takes some 40 vector instructions.)
__device__ inline int udiv_small(int a, int b) {
  int q = (int)((float)a * __builtin_amdgcn_rcpf((float)b));
  const int r = a - q * b;
  q += r >= b ? 1 : 0;
  q -= r < 0 ? 1 : 0;
  return q;
}

// udiv_small of wavefront-uniform operands, its result kept in a scalar
// register
__device__ inline int udiv_uniform(int a, int b) {
  return __builtin_amdgcn_readfirstlane(udiv_small(a, b));
}

// floor(a / b) for a >= 0, b >= 1: the small-operand division where its
// range holds (a branch that is uniform when the operands are), else the
// integer division
__device__ inline int udiv_fast(int a, int b) {
  return ((unsigned)a < (1u << 22) && (unsigned)(b - 1) < (1u << 11) - 1) ? udiv_small(a, b) : a / b;
}

// A thread's walk over the cells of an ex x ey x (ez) box in x-fastest order,
// from linear index c0 in strides of `stride`: one set of divisions at the
// start, then additions with at most one carry per dimension.  A thread whose
// c0 is at or past lim has no cell and skips the divisions.  For boxes that
// fit a workgroup's LDS: c0 and stride below 2^22, ex * ey below 2^11.
struct Walk3 {
  int i, j, k, di, dj, dk, ex, ey;
  __device__ Walk3(int c0, int stride, int ex_, int ey_, int lim = 0x7fffffff)
      : i(0), j(0), k(0), di(0), dj(0), dk(0), ex(max(ex_, 1)), ey(max(ey_, 1)) {
    if (c0 >= lim) return;
    const int exy = ex * ey;  // an empty box walks a 1 x 1 plane and is never read
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

__host__ __device__ inline Geo global_geo(int n) {
  Geo G;
  G.n = n; G.S = 1; G.g = n; G.J = 0; G.m = n; G.ghost = 0;
  G.sstride = (long long)n * n * n;
  return G;
}

__host__ __device__ inline Geo segment_geo(int n, int S, int J) {
  Geo G;
  G.n = n; G.S = S; G.g = n / S; G.J = J;
  G.m = ((G.g + 2 * J) < n ? (G.g + 2 * J) : n) + 2;
  G.ghost = 1;
  G.sstride = (long long)G.m * G.m * G.m;
  return G;
}

// box of segment q (q is ignored on a global level)
__host__ __device__ inline Box seg_box(const Geo& G, int q) {
  Box B;
  int s = (G.S > 1) ? q : 0;
  int p[3] = {s % G.S, (s / G.S) % G.S, s / (G.S * G.S)};
  for (int d = 0; d < 3; ++d) {
    int a = p[d] * G.g - G.J, b = (p[d] + 1) * G.g + G.J;
    B.a[d] = a < 0 ? 0 : a;
    B.b[d] = b > G.n ? G.n : b;
    B.o[d] = B.a[d] - G.ghost;
  }
  B.base = (long long)s * G.sstride;
  return B;
}

// seg_box in device code with the small-operand division (at most 40
// segments per dimension: S^3 below 2^22, S^2 below 2^11)
__device__ inline Box seg_box_d(const Geo& G, int q) {
  Box B;
  const int s = (G.S > 1) ? q : 0;
  const int sy = udiv_uniform(s, G.S), sz = udiv_uniform(sy, G.S);
  const int p[3] = {s - sy * G.S, sy - sz * G.S, sz};
  for (int d = 0; d < 3; ++d) {
    int a = p[d] * G.g - G.J, b = (p[d] + 1) * G.g + G.J;
    B.a[d] = a < 0 ? 0 : a;
    B.b[d] = b > G.n ? G.n : b;
    B.o[d] = B.a[d] - G.ghost;
  }
  B.base = (long long)s * G.sstride;
  return B;
}

__host__ __device__ inline long long at(const Geo& G, const Box& B, int i, int j, int k) {
  return B.base + ((long long)(k - B.o[2]) * G.m + (j - B.o[1])) * G.m + (i - B.o[0]);
}

__host__ __device__ inline bool in_dom(int n, int i, int j, int k) {
  return (unsigned)i < (unsigned)n && (unsigned)j < (unsigned)n && (unsigned)k < (unsigned)n;
}

}  // namespace fmg
