// kernels_descend.hpp -- residual and restriction as one streaming pass.
//
// The first half of the FAS coarse-grid step (Fig. 1; Fig. 6 for segments):
// for every coarse cell of the target region
//   uc = R u             (mean of the 8 children: the solution restriction)
//   rc = R (rhs - L_h u) (mean of the children's residuals).
// A workgroup owns a tile of coarse columns and a chunk of coarse planes; its
// threads own the fine columns under the tile plus a one-cell halo and march
// up the fine planes, holding three planes of u in registers.  The in-plane
// neighbours of the plane being reduced are exchanged through LDS; the
// residuals of the two fine planes of a coarse plane are summed per column
// and the four columns of each coarse cell are then summed from LDS.  Every
// fine value is read once per tile (plus the halo), with whole rows per wave.
//
// mode 0: target = C_fine / 2 of segment q (F of the coarse segment; the
//         whole coarse level on a global level);
// mode 1: target = the genuine coarse cells of segment q, written into the
//         global coarse level (owner computes, at the transition level).
#pragma once
#include "grid.hpp"

namespace fmg {

constexpr int kDescThreads = 1024;

template <class T>
struct DescArgs {
  const T* u;
  Geo gu;
  const T* rhs;
  Geo gr;
  T* uc;
  T* rc;
  Geo gc;
  int mode;
  int ctx, cty, kc;   // coarse tile extent in x, y and coarse planes per chunk
  int ntx, nty, ntz;  // tiles per dimension of the target region
  int nxcd;           // blocks are dealt to this many L2 domains in turn
};

// target coarse box of segment q
__host__ __device__ inline void desc_target(const Geo& gu, const Geo& gc, int q, int mode,
                                            int lo[3], int hi[3]) {
  const Box B = seg_box_d(gu, q);
  if (mode == 0) {
    for (int d = 0; d < 3; ++d) {
      lo[d] = B.a[d] / 2;
      hi[d] = B.b[d] / 2;
    }
  } else {
    const int S = gu.S, e = udiv_small(gc.n, S);  // at most 40 segments per dimension
    const int qy = udiv_small(q, S), qz = udiv_small(qy, S);
    const int p[3] = {q - qy * S, qy - qz * S, qz};
    for (int d = 0; d < 3; ++d) {
      lo[d] = p[d] * e;
      hi[d] = (p[d] + 1) * e;
    }
  }
}

template <class T, int RY, int PF>
__global__ void __launch_bounds__(kDescThreads) __attribute__((amdgpu_waves_per_eu(8)))
k_descend_z(DescArgs<T> a) {
  constexpr int NT = kDescThreads, NC = NT * RY;
  __shared__ T lu[2][NC];              // in-plane exchange, alternating per plane
  __shared__ double lsu[NC], lsr[NC];  // per-column sums over a coarse plane's two fine planes

  const Geo gu = a.gu;
  const int q = blockIdx.y;
  const int n = gu.n;
  const Box B = seg_box_d(gu, q), Br = seg_box_d(a.gr, q), Bc = seg_box_d(a.gc, q);
  int lo[3], hi[3];
  desc_target(gu, a.gc, q, a.mode, lo, hi);

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
  const int I0 = lo[0] + ti * a.ctx, J0 = lo[1] + tj * a.cty, K0 = lo[2] + tk * a.kc;
  if (I0 >= hi[0] || J0 >= hi[1] || K0 >= hi[2]) return;
  const int I1 = I0 + a.ctx < hi[0] ? I0 + a.ctx : hi[0];
  const int J1 = J0 + a.cty < hi[1] ? J0 + a.cty : hi[1];
  const int K1 = K0 + a.kc < hi[2] ? K0 + a.kc : hi[2];
  const int fw = 2 * a.ctx + 2, fh = 2 * a.cty + 2;  // fine tile with its halo
  const long long mm = (long long)gu.m * gu.m;
  const long long rmm = (long long)a.gr.m * a.gr.m;
  const T* __restrict__ ub = a.u + B.base;
  const T* __restrict__ rb = a.rhs + Br.base;
  const double s2 = (double)n * (double)n;

  int ci[RY], uo[RY], ro[RY];
  unsigned fl[RY];  // bit0 u loaded, bit1 residual formed, bit2 coarse owner, bits 4-6 faces
#pragma unroll
  for (int r = 0; r < RY; ++r) {
    const int c = threadIdx.x + NT * r;
    const bool col = c < fw * fh;
    const int cy = udiv_fast(c, fw), cx = c - cy * fw;
    const int x = 2 * I0 - 1 + cx, y = 2 * J0 - 1 + cy;
    // the footprint is x in [2 I0 - 1, 2 I1], y likewise (inside the storage
    // box: C plus its ghost layer); columns past a clipped tile stay idle
    const bool ld = col && x >= 0 && x < n && y >= 0 && y < n && x <= 2 * I1 && y <= 2 * J1;
    const bool res = col && cx >= 1 && cy >= 1 && x < 2 * I1 && y < 2 * J1;
    const bool own = res && ((cx - 1) & 1) == 0 && ((cy - 1) & 1) == 0;
    const unsigned nbxy = (x == 0) + (x == n - 1) + (y == 0) + (y == n - 1);
    fl[r] = (ld ? 1u : 0u) | (res ? 2u : 0u) | (own ? 4u : 0u) | (nbxy << 4);
    ci[r] = col ? c : NC - 1;  // idle slots write a cell no tile column uses
    uo[r] = ld ? (y - B.o[1]) * gu.m + (x - B.o[0]) : 0;
    ro[r] = res ? (y - Br.o[1]) * a.gr.m + (x - Br.o[0]) : 0;
  }

  // loads of plane p: u on every loaded column, rhs on residual columns when
  // p is a plane of the chunk; issued unconditionally, masked at use.  PF
  // planes are in flight.
  const int z0 = 2 * K0 - 1, z1 = 2 * K1;  // fine planes read
  T Qu[PF][RY], Qf[PF][RY];
  unsigned Vu[PF], Vf[PF];
  auto fetch = [&](int p, T(&qu)[RY], T(&qf)[RY], unsigned& vu, unsigned& vf) {
    const bool zu = p >= 0 && p < n && p <= z1;
    const bool zf = p >= 2 * K0 && p < 2 * K1;
    const long long pu = (long long)(p - B.o[2]) * mm;
    const long long pr = (long long)(p - Br.o[2]) * rmm;
    vu = 0;
    vf = 0;
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      const bool v = zu && (fl[r] & 1u);
      const bool w = zf && (fl[r] & 2u);
      vu |= (v ? 1u : 0u) << r;
      vf |= (w ? 1u : 0u) << r;
      qu[r] = ub[v ? pu + uo[r] : 0];
      qf[r] = rb[w ? pr + ro[r] : 0];
    }
  };

  T Ua[RY], Ub[RY], Uc[RY], Fb[RY], Fc[RY];  // planes p-2, p-1, p and rhs of p-1, p
  double su[RY], sr[RY];
#pragma unroll
  for (int r = 0; r < RY; ++r) {
    Ua[r] = Ub[r] = Uc[r] = Fb[r] = Fc[r] = (T)0;
    su[r] = sr[r] = 0.0;
  }
#pragma unroll
  for (int k = 0; k < PF; ++k) fetch(z0 + k, Qu[k], Qf[k], Vu[k], Vf[k]);
  // steps p = z0 .. z1 + 1, padded to a multiple of PF (padding steps reduce nothing)
  const int nsteps = ((z1 + 2 - z0) + PF - 1) / PF * PF;
  for (int pb = z0; pb < z0 + nsteps; pb += PF) {
#pragma unroll
    for (int k = 0; k < PF; ++k) {
      const int p = pb + k;
#pragma unroll
      for (int r = 0; r < RY; ++r) {
        Ua[r] = Ub[r];
        Ub[r] = Uc[r];
        Fb[r] = Fc[r];
        Uc[r] = ((Vu[k] >> r) & 1u) ? Qu[k][r] : (T)0;
        Fc[r] = ((Vf[k] >> r) & 1u) ? Qf[k][r] : (T)0;
      }
      fetch(p + PF, Qu[k], Qf[k], Vu[k], Vf[k]);
      const int zm = p - 1;  // plane reduced in this step
      if (zm >= 2 * K0 && zm < 2 * K1) {  // uniform over the block
        const int b = zm & 1;
#pragma unroll
        for (int r = 0; r < RY; ++r) lu[b][ci[r]] = Ub[r];
        __syncthreads();
        const unsigned nbz = (zm == 0) + (zm == n - 1);
#pragma unroll
        for (int r = 0; r < RY; ++r) {
          if (fl[r] & 2u) {
            const int c = ci[r];
            const double s = (((double)lu[b][c - 1] + (double)lu[b][c + 1]) +
                              ((double)lu[b][c - fw] + (double)lu[b][c + fw])) +
                             ((double)Ua[r] + (double)Uc[r]);
            const double uv = (double)Ub[r];
            const double nb = (double)(6 + ((fl[r] >> 4) & 7u) + nbz);
            const double res = (double)Fb[r] - (s - nb * uv) * s2;
            su[r] = b ? su[r] + uv : uv;
            sr[r] = b ? sr[r] + res : res;
          }
        }
        if (b) {  // second fine plane of coarse plane zm / 2: reduce the 2x2 columns
#pragma unroll
          for (int r = 0; r < RY; ++r) {
            lsu[ci[r]] = su[r];
            lsr[ci[r]] = sr[r];
          }
          __syncthreads();
          const int K = zm >> 1;
#pragma unroll
          for (int r = 0; r < RY; ++r) {
            if (fl[r] & 4u) {
              const int c = ci[r];
              const int cy = udiv_fast(c, fw), cx = c - cy * fw;
              const int I = I0 + ((cx - 1) >> 1), J = J0 + ((cy - 1) >> 1);
              const double tu = (lsu[c] + lsu[c + 1]) + (lsu[c + fw] + lsu[c + fw + 1]);
              const double tr = (lsr[c] + lsr[c + 1]) + (lsr[c + fw] + lsr[c + fw + 1]);
              const long long id = at(a.gc, Bc, I, J, K);
              a.uc[id] = (T)(tu / 8.0);
              a.rc[id] = (T)(tr / 8.0);
            }
          }
        }
      }
    }
  }
}

}  // namespace fmg
