// kernels_norms.hpp -- infinity and 2-norms of a grid function by wavefront
// reduction.
//
// The paper reports the infinity norm of the error and of the residual
// f - L_h u (Sec. 7, Figs. 8 and 10).  k_norms forms, per cell of an n^3 grid,
// r = f - L_h u (mode 0, the 7-point operator with the zero Dirichlet ghosts
// of Eq. 2), r = f - u (mode 1) or r = f (mode 2), and reduces max |r| and
// sum r^2: each thread over a grid-stride range, then across the 64 lanes of
// a wavefront with cross-lane exchanges, then across the wavefronts of the
// workgroup in LDS.  Each workgroup writes one partial pair; k_norms_final reduces the
// partials in one workgroup in a fixed order, so results are deterministic
// for a given grid and launch shape.
#pragma once
#include "grid.hpp"
#include "kernels_simple.hpp"

namespace fmg {

constexpr int kNormThreads = 256;
constexpr int kNormMaxBlocks = 1024;  // partial pairs of one reduction, at most

// the larger of a and b, and NaN when either is NaN (a NaN residual must not
// read as a zero norm)
__device__ inline double max_nan(double a, double b) { return (a > b || a != a) ? a : b; }

__device__ inline void wave_reduce(double& mx, double& ss) {
  for (int off = 32; off > 0; off >>= 1) {
    const double om = __shfl_xor(mx, off, 64);
    const double os = __shfl_xor(ss, off, 64);
    mx = max_nan(om, mx);
    ss += os;
  }
}

// block-wide reduction; the result is valid in thread 0
__device__ inline void block_reduce(double& mx, double& ss) {
  __shared__ double smx[kNormThreads / 64], sss[kNormThreads / 64];
  wave_reduce(mx, ss);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) {
    smx[w] = mx;
    sss[w] = ss;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < (int)(blockDim.x >> 6); ++i) {
      mx = max_nan(smx[i], mx);
      ss += sss[i];
    }
  }
}

__global__ void __launch_bounds__(kNormThreads) k_norms(const double* __restrict__ f,
                                                        const double* __restrict__ u, int n,
                                                        int mode, double* __restrict__ part) {
  const Geo G = global_geo(n);
  const Box B = seg_box(G, 0);
  const long long cnt = (long long)n * n * n;
  double mx = 0.0, ss = 0.0;
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < cnt;
       c += (long long)gridDim.x * blockDim.x) {
    double r;
    if (mode == 0) {
      const int x = (int)(c % n), y = (int)((c / n) % n), z = (int)(c / ((long long)n * n));
      r = f[c] - apply_L<double, double>(u, G, B, x, y, z);
    } else {
      r = mode == 1 ? f[c] - u[c] : f[c];
    }
    mx = max_nan(fabs(r), mx);
    ss += r * r;
  }
  block_reduce(mx, ss);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = mx;
    part[2 * blockIdx.x + 1] = ss;
  }
}

// out[0] = max, out[1] = sqrt(h^3 * sum) with h = 1 / n
__global__ void __launch_bounds__(kNormThreads) k_norms_final(const double* __restrict__ part,
                                                              int nb, int n,
                                                              double* __restrict__ out) {
  double mx = 0.0, ss = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) {
    mx = max_nan(part[2 * i], mx);
    ss += part[2 * i + 1];
  }
  block_reduce(mx, ss);
  if (threadIdx.x == 0) {
    const double h = 1.0 / (double)n;
    out[0] = mx;
    out[1] = sqrt(h * h * h * ss);
  }
}

}  // namespace fmg
