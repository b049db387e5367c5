// kernels_fused.hpp -- temporally blocked red-black Gauss-Seidel smoother and
// a streaming FMG interpolation.
//
// k_smooth_z applies NS half-sweeps (NS/2 red-black sweeps, red first) to the
// compute region C of every segment of a level in one pass over HBM:
//
//  * a workgroup owns an xy tile of txw x tyw columns (chosen per level to fit
//    the compute regions with little waste; RY columns per thread) and
//    marches through a z chunk;
//  * the planes of the z window live in registers: at step p the thread holds
//    plane p, and half-sweep s (s = 1..NS) updates plane p - s, so the NS
//    half-sweeps run as a wavefront in z;
//  * loads run PF planes ahead of use through a ring of registers (the step
//    loop is unrolled PF times), so memory latency overlaps the LDS work of
//    the steps in between; loads are issued unconditionally so the compiler
//    can count them;
//  * x and y neighbours are exchanged through LDS (one barrier per stage);
//  * tiles overlap by NS cells in x and y and a chunk starts NS planes early:
//    the halo is recomputed instead of exchanged, so after NS stages the inner
//    tile and chunk are exact;
//  * u is read from one copy and written to the other: neighbouring tiles
//    overlap, so an in-place update would let a tile read halo cells that its
//    neighbour has already advanced.  Every stored cell inside the domain is
//    written (GSR ghosts unchanged), so the written copy is complete;
//  * in place (inplace = 1) when one workgroup holds a whole segment (one
//    tile covering C plus the halo, one z chunk): segments own their storage
//    and each plane is read before it is written, so nothing else can see a
//    partial update.  Only C is written -- and, after a correction prologue,
//    the GSR ghosts, whose corrected values are final as they are never
//    smoothed;
//  * the load stage is either u itself or u + P(d) with d = w - t on the
//    coarse level, the coarse-grid correction of Fig. 1 and Fig. 6 of the
//    paper (piecewise-constant prolongation), applied on C and the GSR ghosts
//    alike.
//
// A cell of C gets the same point update as in the single-cell kernel,
// u_c = (sum of in-domain neighbours - h^2 rhs_c) / (6 + b_c), with the
// division replaced by a product with the precomputed 1 / (6 + b_c).
#pragma once
#include <type_traits>
#include "grid.hpp"
#include "kernels_simple.hpp"

namespace fmg {

enum { PRO_LOAD = 0, PRO_INTERP = 1, PRO_CORRECT = 2 };

template <class T>
struct SmoothArgs {
  const T* uin;  // current u (read)
  T* u;          // the other copy of u (written)
  Geo gu;
  const T* rhs;
  Geo gr;
  const T* c;   // coarse w (correct: the increment is w - t), or coarse u (interpolation)
  const T* ct;  // coarse t (correct)
  Geo gc;
  T h2;
  int txw, tyw;       // tile extent in x and y (columns, halo included)
  int ntx, nty, ntz;  // tiles per dimension of the write region
  int zc;             // planes per z chunk
  int nxcd;           // blocks are dealt to this many L2 domains in turn
  int inplace;        // 1: one workgroup per segment, u updated in place
  // output epilogue (in place only): the genuine cells go to out (n^3, the
  // caller's FP64 solution) -- written (1) or added (2) -- instead of u
  double* out;
  int outmode;
  // residual-restriction epilogue (RES kernels; k_smooth_z: in place only,
  // k_smooth_cols: two copies on global levels, rmode 0): uc = R u and
  // rc = R (rhs - L u) on the coarse target -- rmode 0: C / 2 of the segment
  // (coarse segment storage); 1: the genuine coarse cells (global level)
  int rmode;
  T* uc;
  T* rc;
  Geo gcr;
  // FAS prologue (load prologue; k_smooth_cols, and k_smooth_z over two
  // copies): rhs holds R res of the level above; the pass forms
  // rhs = R res + L u (Eq. 4) and uses it, and stores it to rhsw and t = u
  // to tw on its output cells
  int fas;
  T* rhsw;
  T* tw;
};

template <class T, int NS, int PRO, int NT, int RY, int PF, int WPE, int RES, int FAS = 0>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(WPE)))
k_smooth_z(SmoothArgs<T> a) {
  constexpr int NC = NT * RY;
  static_assert(PRO == PRO_LOAD || PRO == PRO_CORRECT || PRO == PRO_INTERP, "prologue");
  static_assert(!RES || PRO == PRO_LOAD, "the epilogue follows a load prologue");
  static_assert(!FAS || (PRO == PRO_LOAD && !RES), "the FAS prologue is a plain load pass's");
  // neighbour exchange: per step parity, the idle class of the NS planes the
  // step's stages update (rank-indexed, see below)
  __shared__ T lds[2][NS][NC / 2];
  // epilogue: exchange of the plane being reduced (per step parity: the
  // previous step's is the plane below), each column's rhs of that plane, and
  // per-column sums over the two fine planes of a coarse plane, per coarse
  // plane parity (indexed by slot: each half holds one class by rank, as in
  // the stages)
  __shared__ T ldsr[RES ? 2 : 1][RES ? NC : 1];
  __shared__ T lsf[RES ? NC : 1];
  __shared__ T invd[8];  // 1 / (6 + nb) for nb = 0..6 boundary faces
  // interpolation and correction prologues: the coarse plane under the tile
  // (u, or w - t), per step parity
  __shared__ T lci[PRO != PRO_LOAD ? 2 : 1][PRO != PRO_LOAD ? NT : 1];
  __shared__ double lsu[RES ? 2 : 1][RES ? NC : 1], lsr[RES ? 2 : 1][RES ? NC : 1];
  // FAS prologue: per step parity, the updated class of plane p - 1 before
  // any half-sweep (the idle class is in the exchange), by rank
  __shared__ T lfa[FAS ? 2 : 1][FAS ? NC / 2 : 1];

  const Geo gu = a.gu;
  const int q = blockIdx.y;
  const Box B = seg_box_d(gu, q);
  const int n = gu.n;
  const bool inpl = a.inplace != 0;
  // tile halo: NS columns; a residual over two copies needs the neighbours of
  // the output columns final too, one more
  const int H = NS + ((RES && !inpl) ? 1 : 0);
  const int txw = a.txw, tyw = a.tyw, sx = txw - 2 * H, sy = tyw - 2 * H;
  // blocks are dealt round-robin to the L2 domains: give each domain a
  // contiguous range of tiles so neighbouring tiles share an L2
  int tid = blockIdx.x;
  {
    int nt = a.ntx * a.nty * a.ntz;
    int per = udiv_fast(nt + a.nxcd - 1, a.nxcd);
    const int tq = udiv_fast(tid, a.nxcd);
    int t2 = (tid - tq * a.nxcd) * per + tq;
    if (t2 >= nt) return;
    tid = t2;
  }
  const int tq1 = udiv_fast(tid, a.ntx), tk = udiv_fast(tq1, a.nty);
  const int ti = tid - tq1 * a.ntx, tj = tq1 - tk * a.nty;

  // load region: every stored cell inside the domain.  The tiles partition
  // the load region (two copies) or C (in place); in place, a correction
  // also stores the ghost layer around C.
  int wlo[3], whi[3], glo[3], ghi[3];
  for (int d = 0; d < 3; ++d) {
    wlo[d] = B.o[d] < 0 ? 0 : B.o[d];
    whi[d] = B.o[d] + gu.m > n ? n : B.o[d] + gu.m;
    glo[d] = B.a[d] - 1 < 0 ? 0 : B.a[d] - 1;
    ghi[d] = B.b[d] + 1 > n ? n : B.b[d] + 1;
  }
  // genuine region of the segment (output epilogue)
  const int S = gu.S;
  const int qy = udiv_uniform(q, S), qz = udiv_uniform(qy, S);  // at most 40 segments per dimension
  const int gx0 = (q - qy * S) * gu.g, gy0 = (qy - qz * S) * gu.g, gz0 = qz * gu.g;
  const int tx0 = inpl ? B.a[0] : wlo[0], ty0 = inpl ? B.a[1] : wlo[1];
  const int tz0 = inpl ? B.a[2] : wlo[2], tz1 = inpl ? B.b[2] : whi[2];
  const int ox = tx0 + ti * sx, oy = ty0 + tj * sy, oz = tz0 + tk * a.zc;
  if (ox >= (inpl ? B.b[0] : whi[0]) || oy >= (inpl ? B.b[1] : whi[1]) || oz >= tz1) return;
  int oz1 = oz + a.zc < tz1 ? oz + a.zc : tz1;
  const bool ghosts = inpl && PRO != PRO_LOAD;  // the prologue changed the ghosts too
  const int zs0 = ghosts ? glo[2] : oz, zs1 = ghosts ? ghi[2] : oz1;  // planes stored
  const long long mm = (long long)gu.m * gu.m;

  // steps p0..p1, padded to an even count (steps run in pairs): the padding
  // step only touches planes past the chunk, whose results are never stored.
  // The epilogue trails the last plane by two steps (residual, then the
  // coarse cells of the last coarse plane).
  static_assert(PF == 1 || PF == 2, "the step pairs cycle the load ring");
  // (over two copies the residual epilogue's march starts one plane lower, so
  // that the plane below the chunk is final for its residual too)
  // (the correction starts on an even plane and the interpolation on an odd
  // one, one warm-up step earlier if need be, so that the two steps of a pair
  // share a parent plane, or the pair of coarse planes they lie between)
  const int p00 = oz - NS - ((RES && !inpl) ? 1 : 0);
  const int p0 = PRO == PRO_CORRECT ? (p00 & ~1) : PRO == PRO_INTERP ? ((p00 - 1) | 1) : p00;
  const int p1 = zs1 - 1 + NS + 2 * RES;
  const int nsteps = ((p1 - p0 + 1) + 1) / 2 * 2;

  const Box Br = seg_box_d(a.gr, q);
  const Box Bc = seg_box_d(a.gc, q);
  T* __restrict__ wb = a.u + B.base;
  const T* __restrict__ ub = a.uin + B.base;
  const T* __restrict__ rb = a.rhs + Br.base;
  const T* __restrict__ cd = PRO != PRO_LOAD ? a.c + Bc.base : nullptr;
  const T* __restrict__ cdt = PRO == PRO_CORRECT ? a.ct + Bc.base : nullptr;
  const long long rmm = (long long)a.gr.m * a.gr.m;
  const long long cmm = (long long)a.gc.m * a.gc.m;

  // tile columns are numbered row-major over txw x tyw; thread t owns
  // columns t, t + NT, ...
  // windows: U[j] holds plane p - j, F[j] the rhs of plane p - j (the
  // epilogue, which reduces plane p - NS - 1, takes the plane below and the
  // rhs from LDS)
  constexpr int NU = NS + 2, NF = NS + 1;
  T U[NU][RY], F[NF][RY];
  // FAS prologue: plane p - 2 as loaded (half-sweeps have changed U[2])
  T Uo[FAS ? RY : 1];
  T Qu[PF][RY], Qf[PF][RY];  // ring of planes in flight
  // interpolation prologue: this thread's coarse value of a fetched coarse
  // plane in the ring, and the xy-interpolated coarse planes lo and lo + 1 of
  // the current fine plane (lo = floor((p - 1) / 2))
  // (the correction prologue: this thread's w and t of the parent plane)
  T Qi[PF], Qj[PF], clo[RY], chi[RY];
  // Columns are dealt to thread slots sorted by colour class: slots
  // [0, NC/2) hold the columns of one (x + y) parity, slots [NC/2, NC) the
  // other (txw is even, so every row has txw/2 of each).  In a half-sweep only
  // one class has the colour being updated, so whole wavefronts (RY = 1) or
  // whole slots (RY = 2) are active or idle together, and no lane computes a
  // cell it then discards.  The half [NC/2, NC) holds parity c0 ^ 1 with
  // c0 = (p0 - 1) & 1: every stage of step p0 + j updates parity (p - 1) & 1
  // (see the step), which is then the class of half j & 1.
  // A column's rank in its class is i = cy txw/2 + cx/2; the exchange holds
  // one class per plane indexed by rank, so a wavefront's LDS accesses are
  // unit stride (no bank conflicts).  The in-plane neighbours of a column are
  // in the other class, at ranks i - 1 + (cx & 1), i + (cx & 1) (x) and
  // i -+ txw/2 (y).
  int xr[RY], ys[RY], uo[RY];
  const int c0 = (p0 - 1) & 1;
  // half and rank of slot r
  auto kbh = [&](int r) -> int { return threadIdx.x + NT * r >= NC / 2 ? 1 : 0; };
  auto rnk = [&](int r) -> int {
    const int sl = threadIdx.x + NT * r;
    return sl >= NC / 2 ? sl - NC / 2 : sl;
  };
  bool lact[RY];  // the slot's column is updated (inside C, not a tile edge)
  // 1 / (6 + x and y boundary faces) of the slot's column: the diagonal inverse
  // of the steps whose planes all lie off the z walls (INNER), without LDS
  T invr[RY];
  // interpolation and correction prologues: the tile's threads load the
  // coarse columns under the tile, ctx x cty from (cX0, cY0), one each, into
  // LDS.  Per slot: the LDS index of the coarse column (X0, Y0) under its
  // column and, for the interpolation, in ok bits 10-13, where X1 / Y1 lie:
  // next (odd x / y) or previous, or reflected at a wall (X1 = X0, sign -1)
  const int cX0 = ((ox - H) >> 1) - 1, cY0 = ((oy - H) >> 1) - 1;
  const int ctx = (txw >> 1) + 3, ctn = ctx * ((tyw >> 1) + 3);
  int tco = 0;  // this thread's coarse column (offset in the coarse box), if any
  bool tcv = false;
  if (PRO != PRO_LOAD && (int)threadIdx.x < ctn) {
    const int tyq = udiv_small((int)threadIdx.x, ctx);  // ctx <= 131
    const int X = cX0 + (int)threadIdx.x - tyq * ctx, Y = cY0 + tyq;
    tcv = X >= 0 && X < a.gc.n && Y >= 0 && Y < a.gc.n && X >= Bc.o[0] && X < Bc.o[0] + a.gc.m &&
          Y >= Bc.o[1] && Y < Bc.o[1] + a.gc.m;
    tco = tcv ? (Y - Bc.o[1]) * a.gc.m + (X - Bc.o[0]) : 0;
  }
  int io[PRO != PRO_LOAD ? RY : 1];
  unsigned ok[RY];  // bit0 stored xy, bit1 in C xy, bit2 output xy, bit3 not tile edge,
                    // bits 4-6 boundary faces in x and y, bit7 genuine, bit8 owns a
                    // coarse column (epilogue), bit9 cx odd
#pragma unroll
  for (int r = 0; r < RY; ++r) {
    const int sl = threadIdx.x + NT * r;
    const int h = sl >= NC / 2 ? 1 : 0, i = sl - h * (NC / 2), tw2 = txw >> 1, k = h ^ c0;
    const bool col = i < tw2 * tyw;
    const int cy = col ? udiv_small(i, tw2) : 0;  // tw2 <= 128
    // (x + y) parity of the tile column (cx, cy) is (ox + oy + cx + cy) & 1
    const int cx = col ? 2 * (i - cy * tw2) + ((cy + k + ox + oy) & 1) : 0;
    const int x = ox - H + cx, y = oy - H + cy;
    xr[r] = x;
    ys[r] = y;
    const bool st = col && x >= wlo[0] && x < whi[0] && y >= wlo[1] && y < whi[1];
    const bool inc = col && x >= B.a[0] && x < B.b[0] && y >= B.a[1] && y < B.b[1];
    const bool ing = col && x >= glo[0] && x < ghi[0] && y >= glo[1] && y < ghi[1];
    const bool outp = inpl ? (inc || (ghosts && ing))
                           : (st && cx >= H && cx < txw - H && cy >= H && cy < tyw - H);
    const bool inner = col && cx > 0 && cx < txw - 1 && cy > 0 && cy < tyw - 1;
    const unsigned nbxy = (x == 0) + (x == n - 1) + (y == 0) + (y == n - 1);
    const bool gen = col && x >= gx0 && x < gx0 + gu.g && y >= gy0 && y < gy0 + gu.g;
    // epilogue: the column holding child (0,0) of a coarse target cell (the
    // output columns are C in place)
    const bool own = RES && (a.rmode == 0 ? outp && ((x - B.a[0]) & 1) == 0 && ((y - B.a[1]) & 1) == 0
                                          : gen && (x & 1) == 0 && (y & 1) == 0);
    ok[r] = (st ? 1u : 0u) | (inc ? 2u : 0u) | (outp ? 4u : 0u) | (inner ? 8u : 0u) | (nbxy << 4) |
            (gen ? 128u : 0u) | (own ? 256u : 0u) | ((unsigned)(cx & 1) << 9);
    lact[r] = inc && inner;
    invr[r] = (T)1 / (T)(6 + (int)nbxy);
    if (PRO != PRO_LOAD) {
      const int nc = a.gc.n, X0 = x >> 1, Y0 = y >> 1;
      const int X1 = (x & 1) ? X0 + 1 : X0 - 1, Y1 = (y & 1) ? Y0 + 1 : Y0 - 1;
      const bool rx = X1 < 0 || X1 >= nc, ry = Y1 < 0 || Y1 >= nc;
      // stored columns lie one coarse column inside the coarse tile on each side
      io[r] = st ? (Y0 - cY0) * ctx + (X0 - cX0) : ctx + 1;
      if (PRO == PRO_INTERP)
        ok[r] |= ((unsigned)(x & 1) << 10) | (rx ? 1u << 11 : 0u) | ((unsigned)(y & 1) << 12) |
                 (ry ? 1u << 13 : 0u);
    }
    uo[r] = (y - B.o[1]) * gu.m + (x - B.o[0]);
#pragma unroll
    for (int j = 0; j < NU; ++j) U[j][r] = 0;
#pragma unroll
    for (int j = 0; j < NF; ++j) F[j][r] = 0;
    if (FAS) Uo[r] = 0;
  }

  // issue the loads of plane p into a ring slot (raw values, used PF steps
  // later).  Every load is issued unconditionally -- lanes with nothing to
  // read fetch the first element of the same array and their validity bit
  // masks the value at use -- so loads in flight can be counted exactly.
  unsigned Vu[PF], Vf[PF];
  // interpolation prologue: this thread's load of coarse plane P (reflected at
  // the walls); threads without a coarse column, and planes outside the coarse
  // box, read its first element
  auto fetch_c = [&](int P) -> T {
    if (P < 0) P = -1 - P;
    else if (P >= a.gc.n) P = 2 * a.gc.n - 1 - P;
    const bool v = tcv && P >= Bc.o[2] && P < Bc.o[2] + a.gc.m;
    return cd[v ? (long long)(P - Bc.o[2]) * cmm + tco : 0];
  };
  // ... and the xy interpolation of slot r from the coarse plane in LDS
  // (weights 9, 3, 3, 1 / 16; a reflected neighbour enters with sign -1);
  // flip: the plane itself was reflected
  auto cxy = [&](const T* pl, int r, bool flip) -> T {
    const unsigned f = ok[r];
    const int dx = (f & (1u << 11)) ? 0 : ((f & (1u << 10)) ? 1 : -1);
    const int dy = (f & (1u << 13)) ? 0 : ((f & (1u << 12)) ? ctx : -ctx);
    const int i0 = io[r];
    const T q0 = pl[i0], q1 = pl[i0 + dx], q2 = pl[i0 + dy], q3 = pl[i0 + dx + dy];
    const T s1 = (f & (1u << 11)) ? -q1 : q1;
    const T s2 = (f & (1u << 13)) ? -q2 : q2;
    const T s3 = (((f >> 11) ^ (f >> 13)) & 1u) ? -q3 : q3;
    const T c = (T)0.5625 * q0 + ((T)0.1875 * (s1 + s2) + (T)0.0625 * s3);
    return flip ? -c : c;
  };
  auto fetch = [&](int p, T(&qu)[RY], T(&qf)[RY], T& qi, T& qj, unsigned& vu, unsigned& vf,
                   bool ldc) {
    if (PRO == PRO_INTERP && ldc) qi = fetch_c(((p - 1) >> 1) + 1);  // odd planes only
    // w and t of the parent plane (no reflection: parents lie inside), for
    // even planes only: fine planes 2P and 2P + 1 share it (ldc is a
    // compile-time fact of the step that fetches)
    if (PRO == PRO_CORRECT && ldc) {
      const int P = p >> 1;
      const bool v = tcv && P >= Bc.o[2] && P < Bc.o[2] + a.gc.m;
      const long long ic = v ? (long long)(P - Bc.o[2]) * cmm + tco : 0;
      qi = cd[ic];
      qj = cdt[ic];
    }
    const bool zs = p >= wlo[2] && p < whi[2];
    const bool zcin = p >= B.a[2] && p < B.b[2];
    const long long pu = (long long)(p - B.o[2]) * mm;
    const long long pr = (long long)(p - Br.o[2]) * rmm;
    vu = 0;
    vf = 0;
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      const bool v = zs && (ok[r] & 1u);
      const bool w = v && zcin && (ok[r] & 2u);
      vu |= (v ? 1u : 0u) << r;
      vf |= (w ? 1u : 0u) << r;
      if (PRO != PRO_INTERP) qu[r] = ub[v ? pu + uo[r] : 0];
      qf[r] = rb[w ? pr + (ys[r] - Br.o[1]) * a.gr.m + (xr[r] - Br.o[0]) : 0];
    }
  };

  if (threadIdx.x < 7) invd[threadIdx.x] = (T)1 / (T)(6 + (int)threadIdx.x);  // read after a barrier
  if constexpr (PRO == PRO_INTERP) {  // the window starts with lo(p0) in both planes
    const int lo = (p0 - 1) >> 1;
    if ((int)threadIdx.x < ctn) lci[1][threadIdx.x] = fetch_c(lo);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RY; ++r) clo[r] = chi[r] = cxy(lci[1], r, lo < 0 || lo >= a.gc.n);
  }
#pragma unroll
  for (int k = 0; k < PF; ++k) fetch(p0 + k, Qu[k], Qf[k], Qi[k], Qj[k], Vu[k], Vf[k], (k & 1) == 0);
  // step p0 + j with J = j & 1: the stages update the slots of half J
  auto step = [&](auto Jc, int p) {
    constexpr int J = decltype(Jc)::value, kq = J % PF;
#pragma unroll
    for (int j = NU - 1; j > 0; --j)
#pragma unroll
      for (int r = 0; r < RY; ++r) U[j][r] = U[j - 1][r];
#pragma unroll
    for (int j = NF - 1; j > 0; --j)
#pragma unroll
      for (int r = 0; r < RY; ++r) F[j][r] = F[j - 1][r];
    // U[0] of the interpolation and correction prologues is formed after the
    // exchange, from the coarse plane staged in LDS
    const unsigned vuk = Vu[kq];
    T uq[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      if (PRO == PRO_LOAD) U[0][r] = ((vuk >> r) & 1u) ? Qu[kq][r] : (T)0;
      uq[r] = Qu[kq][r];
      F[0][r] = ((Vf[kq] >> r) & 1u) ? Qf[kq][r] : (T)0;
    }
    // the correction stages w - t once per parent plane P (in the pair's even
    // step, J = 0: p0 is even) in buffer P & 1, which the next write (parent
    // P + 2) reaches two barriers later
    // (the interpolation likewise stages coarse plane lo + 1 once, in the
    // pair's odd step, J = 0: p0 is odd, in a buffer per pair parity)
    const int cbuf = PRO == PRO_CORRECT ? (p >> 1) & 1 : PRO == PRO_INTERP ? ((p - p0) >> 1) & 1 : J;
    if constexpr (PRO == PRO_INTERP && J == 0) {
      if ((int)threadIdx.x < ctn) lci[cbuf][threadIdx.x] = Qi[kq];
    }
    if constexpr (PRO == PRO_CORRECT && J == 0) {
      if ((int)threadIdx.x < ctn) lci[cbuf][threadIdx.x] = Qi[kq] - Qj[kq];
    }
    fetch(p + PF, Qu[kq], Qf[kq], Qi[kq], Qj[kq], Vu[kq], Vf[kq], ((J + PF) & 1) == 0);
    // NS half-sweeps as a wavefront: stage s applies half-sweep s (colour
    // (s - 1) & 1) to plane p - s.  Its cells read the other colour of that
    // plane as the previous step left it (no stage of this step changes it),
    // the plane above from stage s - 1 of this step and the plane below from
    // the previous step (both in this thread's registers).  So one exchange
    // per step serves all stages, and every stage updates the same parity,
    // (p - s + (s - 1)) & 1 = (p - 1) & 1: half J.
#pragma unroll
    for (int s = 1; s <= NS; ++s)
#pragma unroll
      for (int r = 0; r < RY; ++r)
        if (kbh(r) != J) lds[J][s - 1][rnk(r)] = U[s][r];
    if constexpr (RES) {  // the epilogue's plane p - NS - 1 (final since the last step)
#pragma unroll
      for (int r = 0; r < RY; ++r) ldsr[J][threadIdx.x + NT * r] = U[NS + 1][r];
    }
    if constexpr (FAS) {
#pragma unroll
      for (int r = 0; r < RY; ++r)
        if (kbh(r) == J) lfa[J][rnk(r)] = U[1][r];
    }
    __syncthreads();
    if constexpr (FAS) {
      // rhs of plane zf = p - 1 becomes R res + L u (FP64; neighbours summed in
      // the order of the single-cell kernels, out-of-domain ones are the zeros
      // loaded), on every column the half-sweeps update, before the first
      // of them (stage 1 of this step) reads it.  Plane p - 1 and the in-plane
      // neighbours are as loaded; plane p - 2 comes from Uo.
      const int zf = p - 1;
      const bool zin = zf >= 0 && zf < n, zout = zf >= oz && zf < oz1;  // uniform
      const double s2 = (double)n * (double)n;
      const unsigned nbz = (zf == 0) + (zf == n - 1);
      const long long pw = (long long)(zf - B.o[2]) * mm;
#pragma unroll
      for (int r = 0; r < RY; ++r) {
        if (zin && (ok[r] & 10u) == 10u) {  // inside C, not a tile edge: neighbours in the tile
          const T* pl = kbh(r) == J ? lds[J][0] : lfa[J];
          const int tw2 = txw >> 1, i = rnk(r);
          const int xn = i - 1 + (int)((ok[r] >> 9) & 1u);
          double sn = (double)pl[xn];
          sn += (double)pl[xn + 1];
          sn += (double)pl[i - tw2];
          sn += (double)pl[i + tw2];
          sn += (double)Uo[r];
          sn += (double)U[0][r];
          const double nb = (double)(6u + ((ok[r] >> 4) & 7u) + nbz);
          F[1][r] = (T)((double)F[1][r] + (sn - nb * (double)U[1][r]) * s2);
          if (zout && (ok[r] & 4u)) {
            a.rhsw[pw + uo[r]] = F[1][r];
            a.tw[pw + uo[r]] = U[1][r];
          }
        }
        Uo[r] = U[1][r];
      }
    }
    if constexpr (PRO == PRO_CORRECT) {  // u + (w - t) of the parent (Eq. 4's correction, piecewise constant)
#pragma unroll
      for (int r = 0; r < RY; ++r) U[0][r] = ((vuk >> r) & 1u) ? uq[r] + lci[cbuf][io[r]] : (T)0;
    }
    if constexpr (PRO == PRO_INTERP) {
      // plane p lies between coarse planes lo and lo + 1; lo advances on odd
      // p (J = 0), and p takes 3/4 of the nearer one (FMG interpolation:
      // trilinear, odd reflection at the walls); the even plane after it
      // lies between the same two
      if constexpr (J == 0) {
        const int Pn = ((p - 1) >> 1) + 1;
        const bool flip = Pn < 0 || Pn >= a.gc.n;
#pragma unroll
        for (int r = 0; r < RY; ++r) {
          clo[r] = chi[r];
          chi[r] = cxy(lci[cbuf], r, flip);
          const T v = (T)0.75 * clo[r] + (T)0.25 * chi[r];
          U[0][r] = ((vuk >> r) & 1u) ? v : (T)0;
        }
      } else {
#pragma unroll
        for (int r = 0; r < RY; ++r) {
          const T v = (T)0.75 * chi[r] + (T)0.25 * clo[r];
          U[0][r] = ((vuk >> r) & 1u) ? v : (T)0;
        }
      }
    }
    // the stages; INNER: all NS planes lie inside C and off the domain's z
    // walls (most steps), so no stage tests its plane
    auto stages = [&](auto INNERc) {
      constexpr bool INNER = decltype(INNERc)::value;
#pragma unroll
      for (int s = 1; s <= NS; ++s) {
        const int zp = p - s;
        int nbz = 0;
        if constexpr (!INNER) {
          if (zp < B.a[2] || zp >= B.b[2]) continue;  // uniform over the block
          nbz = (zp == 0) + (zp == n - 1);
        }
#pragma unroll
        for (int r = 0; r < RY; ++r) {
          if (kbh(r) != J) continue;  // compile-time for RY = 2, per wavefront for RY = 1
          // every lane of the slot computes; lanes whose column is not updated
          // keep their value
          // the stencil reads around the slot's rank, or around rank tw2 for
          // columns that are never updated, so that every read is in bounds
          const T* pl = lds[J][s - 1];
          const int tw2 = txw >> 1, i = lact[r] ? rnk(r) : tw2;
          const int xn = i - 1 + (int)((ok[r] >> 9) & 1u);
          // the plane above (just updated by stage s - 1) is added last
          const T sum = (((pl[xn] + pl[xn + 1]) + (pl[i - tw2] + pl[i + tw2])) + U[s + 1][r]) +
                        U[s - 1][r];
          const T inv = INNER ? invr[r] : invd[(int)((ok[r] >> 4) & 7u) + nbz];
          const T nv = (sum - a.h2 * F[s][r]) * inv;
          U[s][r] = lact[r] ? nv : U[s][r];
        }
      }
    };
    // (kernels held to 64 registers for two workgroups per CU keep one path)
    if (WPE < 8 && p - NS >= B.a[2] && p - 1 < B.b[2] && p - NS >= 1 && p - 1 <= n - 2)
      stages(std::integral_constant<bool, WPE < 8>{});
    else
      stages(std::false_type{});
    // plane p - NS is final
    const int zo = p - NS;
    if (a.outmode) {  // genuine cells to the caller's solution
      if (zo >= gz0 && zo < gz0 + gu.g) {
#pragma unroll
        for (int r = 0; r < RY; ++r) {
          if (ok[r] & 128u) {
            const long long io = ((long long)zo * n + ys[r]) * n + xr[r];
            a.out[io] = a.outmode == 2 ? a.out[io] + (double)U[NS][r] : (double)U[NS][r];
          }
        }
      }
    } else if (zo >= zs0 && zo < zs1) {
      const long long pw = (long long)(zo - B.o[2]) * mm;
#pragma unroll
      for (int r = 0; r < RY; ++r)
        if (ok[r] & 4u) wb[pw + uo[r]] = U[NS][r];
    }
    // epilogue: residual of plane zr = p - NS - 1 (its neighbours zr +- 1
    // are final), summed over the two fine planes of each coarse plane, then,
    // one step later, over the 2 x 2 columns of each coarse cell.  Every LDS
    // value it reads from other slots was written before this step's
    // exchange barrier: the plane zr in the exchange of parity J, and the
    // sums of coarse plane (zr - 1) / 2, complete at the last step, in the
    // buffer of its parity.  Each is rewritten two steps later at the
    // earliest, after the next step's barrier.
    const int zr = p - NS - 1;
    // slot sl's column at [sl]; pn: the slot of the same rank in the other half
    auto pnb = [&](int r) -> int {
      const int sl = threadIdx.x + NT * r;
      return sl >= NC / 2 ? sl - NC / 2 : sl + NC / 2;
    };
    if constexpr (RES) if (((zr - 1) & 1) && zr - 1 >= oz && zr - 1 < oz1) {
      // coarse plane (zr - 1) / 2 (uniform over the block)
      const int zc = (zr - 1) >> 1, cb = zc & 1;
      const bool zt = a.rmode == 0 || (zr - 1 >= gz0 && zr - 1 < gz0 + gu.g);
      const Box Bo = seg_box_d(a.gcr, q);
#pragma unroll
      for (int r = 0; r < RY; ++r) {
        if (zt && (ok[r] & 256u)) {
          // the 2 x 2 columns (cx, cy) .. (cx + 1, cy + 1): this slot, the
          // other half at ranks + (cx & 1) and + txw/2, and this half at
          // rank + txw/2 + (cx & 1)
          const int sl = threadIdx.x + NT * r, pn = pnb(r), tw2 = txw >> 1;
          const int od = (int)((ok[r] >> 9) & 1u);
          const double* su = lsu[cb];
          const double* sr = lsr[cb];
          const double tu = (su[sl] + su[pn + od]) + (su[pn + tw2] + su[sl + tw2 + od]);
          const double tr = (sr[sl] + sr[pn + od]) + (sr[pn + tw2] + sr[sl + tw2 + od]);
          const long long id = at(a.gcr, Bo, xr[r] >> 1, ys[r] >> 1, zc);
          a.uc[id] = (T)(tu / 8.0);
          a.rc[id] = (T)(tr / 8.0);
        }
      }
    }
    // (the chunk's planes [oz, oz1) are C in place; chunks start on an even plane)
    if constexpr (RES) if (zr >= oz && zr < oz1) {  // uniform over the block
      const unsigned nbz = (zr == 0) + (zr == n - 1);
      const double s2 = (double)n * (double)n;
      const bool odd = zr & 1;
      const int cb = (zr >> 1) & 1;
#pragma unroll
      for (int r = 0; r < RY; ++r) {
        if (ok[r] & 4u) {  // output columns lie H inside the tile: neighbours are in it
          const int sl = threadIdx.x + NT * r, pn = pnb(r), tw2 = txw >> 1;
          const int xn = pn - 1 + (int)((ok[r] >> 9) & 1u);
          const T* pl = ldsr[J];
          // the plane below is this slot's own entry of the previous step
          const double sn = (((double)pl[xn] + (double)pl[xn + 1]) +
                             ((double)pl[pn - tw2] + (double)pl[pn + tw2])) +
                            ((double)ldsr[J ^ 1][sl] + (double)U[NS][r]);
          const double uv = (double)U[NS + 1][r];
          const double nb = (double)(6u + ((ok[r] >> 4) & 7u) + nbz);
          const double res = (double)lsf[sl] - (sn - nb * uv) * s2;
          // the column's sums over the two fine planes, kept in its own LDS entry
          lsu[cb][sl] = odd ? lsu[cb][sl] + uv : uv;
          lsr[cb][sl] = odd ? lsr[cb][sl] + res : res;
        }
      }
    }
    if constexpr (RES) {  // the rhs of plane p - NS, which the next step reduces
#pragma unroll
      for (int r = 0; r < RY; ++r) lsf[threadIdx.x + NT * r] = F[NS][r];
    }
  };
  for (int pb = p0; pb < p0 + nsteps; pb += 2) {
    step(std::integral_constant<int, 0>{}, pb);
    // keep the two steps apart: interleaving them only lengthens live ranges
    __builtin_amdgcn_sched_barrier(0);
    step(std::integral_constant<int, 1>{}, pb + 1);
  }
}

// ---------------------------------------------------------------------------
// FMG interpolation Pi (Sec. 3.2): trilinear with odd reflection at the walls,
// onto every stored cell inside the domain (C and GSR ghosts).  One thread
// per fine column marches a z chunk.  Fine plane z uses the coarse planes lo
// and lo + 1 with lo = floor((z - 1) / 2): child 2P takes 3/4 c(P) + 1/4
// c(P-1), child 2P+1 takes 3/4 c(P) + 1/4 c(P+1).  The xy interpolation of a
// coarse plane (4 loads) is kept while two consecutive fine planes use it, and
// only the planes a fine plane needs are read (they lie in the coarse
// segment's storage when the coarser buffer is at least half as wide).
template <class T>
__global__ void __launch_bounds__(256) k_interp_z(T* __restrict__ u, Geo gu,
                                                  const T* __restrict__ c, Geo gc, int zc, int ce) {
  const int q = blockIdx.y;
  const Box B = seg_box_d(gu, q), Bc = seg_box_d(gc, q);
  const int n = gu.n, nc = gc.n;
  int lo[3], hi[3];
  for (int d = 0; d < 3; ++d) {
    lo[d] = B.o[d] < 0 ? 0 : B.o[d];
    hi[d] = B.o[d] + gu.m > n ? n : B.o[d] + gu.m;
  }
  const int t = blockIdx.x * blockDim.x + threadIdx.x;  // the grid stays below 2^31 threads
  const int t1 = udiv_fast(t, ce), kz = udiv_fast(t1, ce);
  const int cx = t - t1 * ce, cy = t1 - kz * ce;
  const int x = lo[0] + cx, y = lo[1] + cy, z0 = lo[2] + kz * zc;
  if (x >= hi[0] || y >= hi[1] || z0 >= hi[2]) return;
  const int z1 = z0 + zc < hi[2] ? z0 + zc : hi[2];

  // xy stencil of this column: coarse columns (X0|X1, Y0|Y1) and weights
  int X0 = x >> 1, Y0 = y >> 1;
  int X1 = (x & 1) ? X0 + 1 : X0 - 1, Y1 = (y & 1) ? Y0 + 1 : Y0 - 1;
  T sx = 1, sy = 1;
  if (X1 < 0) { X1 = 0; sx = -1; }
  if (X1 >= nc) { X1 = nc - 1; sx = -1; }
  if (Y1 < 0) { Y1 = 0; sy = -1; }
  if (Y1 >= nc) { Y1 = nc - 1; sy = -1; }
  const T w00 = (T)0.5625, w10 = (T)0.1875 * sx, w01 = (T)0.1875 * sy, w11 = (T)0.0625 * sx * sy;
  const T* __restrict__ cb = c + Bc.base;
  const long long cmm = (long long)gc.m * gc.m;
  const int o00 = (Y0 - Bc.o[1]) * gc.m + (X0 - Bc.o[0]);
  const int o10 = (Y0 - Bc.o[1]) * gc.m + (X1 - Bc.o[0]);
  const int o01 = (Y1 - Bc.o[1]) * gc.m + (X0 - Bc.o[0]);
  const int o11 = (Y1 - Bc.o[1]) * gc.m + (X1 - Bc.o[0]);
  // xy-interpolated coarse plane P, odd reflection outside [0, nc)
  auto plane = [&](int P) -> T {
    T sg = 1;
    if (P < 0) { P = -1 - P; sg = -1; }
    if (P >= nc) { P = 2 * nc - 1 - P; sg = -1; }
    const long long pz = (long long)(P - Bc.o[2]) * cmm;
    return sg * (w00 * cb[pz + o00] + w10 * cb[pz + o10] + w01 * cb[pz + o01] +
                 w11 * cb[pz + o11]);
  };
  T* __restrict__ ucol = u + B.base + (long long)(y - B.o[1]) * gu.m + (x - B.o[0]);
  const long long mm = (long long)gu.m * gu.m;
  int lo_p = (z0 - 1) >> 1;
  T clo = plane(lo_p), chi = plane(lo_p + 1);
  for (int z = z0; z < z1; ++z) {
    const int l = (z - 1) >> 1;
    if (l != lo_p) {  // advance by one coarse plane
      lo_p = l;
      clo = chi;
      chi = plane(l + 1);
    }
    T v = (z & 1) ? (T)0.75 * clo + (T)0.25 * chi : (T)0.75 * chi + (T)0.25 * clo;
    ucol[(long long)(z - B.o[2]) * mm] = v;
  }
}

}  // namespace fmg

namespace fmg {

// ---------------------------------------------------------------------------
// Box-resident smoother for segment levels whose whole storage box fits in
// LDS (Sec. 4 of the paper: a segment is processed on its own, with frozen
// ghosts).  One workgroup per segment loads the box (u, or u + P(d) for the
// coarse-grid correction), applies nu red-black sweeps in LDS with a barrier
// between half-sweeps, and writes the box back in place (segments own their
// storage, so no other workgroup reads it meanwhile).  Each thread owns fixed
// pairs of x-adjacent cells, one of each colour, so every thread updates a
// cell in every half-sweep.
constexpr int kBoxThreads = 1024;
constexpr int kBoxSlots = 8;  // cell pairs per thread
// box cells per thread in flight while loading (bounded by registers: the
// slots' right-hand sides are in flight too), fewer with the correction
// prologue (three loads per cell)
constexpr int kBoxLoads = 12;
constexpr int kBoxLoadsCorrect = 6;

template <class T>
struct BoxArgs {
  T* u;
  Geo gu;
  const T* rhs;
  Geo gr;
  const T* d;   // coarse w (correct: the increment is w - t)
  const T* dt;  // coarse t (correct)
  Geo gc;
  T h2;
  int nu;
  // FAS prologue (fas > 0, load prologue only): the level was just restricted
  // into; rhs holds R res on F.  The kernel forms rhs = R res + L u on F and
  // L u on C \ F (Fig. 6; fas == 2: F is the whole region), writes it back
  // over rhs, and writes t = the loaded box where the finer level's
  // correction reads it (the parents of its stored cells).
  int fas;
  T* rhsw;  // = rhs, writable
  T* t;
  Geo gf;   // the finer level: F = its compute region / 2
  // residual-restriction epilogue (rmode >= 0): uc = R u and rc = R (rhs -
  // L u) on the coarse target (rmode 0: C / 2 of the segment; 1: the genuine
  // coarse cells, in the global coarse level)
  int rmode;
  T* uc;
  T* rc;
  Geo gcr;
};

// 1 / (6 + nb) for nb = 0..3 boundary faces, without a division (a cell of
// a level with edge n >= 2 touches at most one wall per dimension)
template <class T>
__device__ inline T box_inv_diag(unsigned nb) {
  const T lo = (nb & 1u) ? (T)(1.0 / 7.0) : (T)(1.0 / 6.0);
  const T hi = (nb & 1u) ? (T)(1.0 / 9.0) : (T)(1.0 / 8.0);
  return (nb & 2u) ? hi : lo;
}

template <class T, int PRO>
__global__ void __launch_bounds__(kBoxThreads) k_smooth_box(BoxArgs<T> a) {
  extern __shared__ unsigned char smem_raw[];
  T* bu = reinterpret_cast<T*>(smem_raw);
  const Geo gu = a.gu;
  const int q = blockIdx.x, n = gu.n, m = gu.m, m2 = m * m, mc = m * m2;
  const int NT = blockDim.x;
  const Box B = seg_box_d(gu, q), Br = seg_box_d(a.gr, q), Bc = seg_box_d(a.gc, q);
  T* __restrict__ ub = a.u + B.base;
  const T* __restrict__ rb = a.rhs + Br.base;
  const bool fas = PRO == PRO_LOAD && a.fas > 0;

  // the load prologue copies the box straight into LDS (global_load_lds, 16
  // bytes per lane, 1 KiB per wavefront instruction, no registers), issued
  // first so that the slot setup overlaps it; cells outside the domain are
  // zeroed once it has landed.  Needs 16-byte alignment of the box and its
  // length.  With an even box edge every row starts 16-byte aligned, and the
  // copy skips the planes and rows outside the domain (boundary segments):
  // per plane inside, one contiguous run of the rows inside.
  const long long bytes = (long long)mc * sizeof(T);
  const bool dma = PRO == PRO_LOAD && ((B.base * (long long)sizeof(T)) & 15) == 0 && (bytes & 15) == 0;
  if (dma) {
    const int nw = NT >> 6, wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
    const char* src = reinterpret_cast<const char*>(ub);
    char* dst = reinterpret_cast<char*>(bu);
    const bool rows = (m & 1) == 0;
    const int zl = rows ? max(0, -B.o[2]) : 0, zh = rows ? min(m, n - B.o[2]) : 1;
    const int yl = rows ? max(0, -B.o[1]) : 0, yh = rows ? min(m, n - B.o[1]) : m;
    // run of plane z: bytes [(z m + yl) m, (z m + yh) m) * sizeof(T); without
    // rows, one run: the whole box
    const long long run = rows ? (long long)(yh - yl) * m * (long long)sizeof(T) : bytes;
    const int cpr = (int)((run + 1023) >> 10);  // chunks per run
    const int nch = (zh - zl) * cpr;
    for (int ch = wv; ch < nch; ch += nw) {
      const int cq = udiv_small(ch, cpr), pz = zl + cq, c = ch - cq * cpr;
      const long long o = ((long long)pz * m + yl) * m * (long long)sizeof(T) + (long long)c * 1024;
      if ((long long)c * 1024 + ln * 16 < run)
        __builtin_amdgcn_global_load_lds(src + o + ln * 16,
                                         (__attribute__((address_space(3))) void*)(dst + o),
                                         16, 0, 0);
    }
  }

  // cell pairs of C: pair (xp, y, z) holds x = a0 + 2 xp and x + 1; the
  // right-hand side and diagonal inverse of both cells stay in registers.
  // Set up first, so that the right-hand side loads overlap the box loads.
  const int cx = B.b[0] - B.a[0], cy = B.b[1] - B.a[1], cz = B.b[2] - B.a[2];
  const int px = (cx + 1) / 2, np = px * cy * cz;
  int li[kBoxSlots], gi[kBoxSlots];
  unsigned fl[kBoxSlots];  // bit0 parity of the first cell, bit1 second cell exists,
                           // bits 2-3 / 4-5 boundary faces of the first / second cell,
                           // bits 6 / 7 first / second cell in F (FAS prologue)
  T r0[kBoxSlots], r1[kBoxSlots];
  int ns = 0;
  int flo[3] = {0, 0, 0}, fhi[3] = {n, n, n};
  if (fas && a.fas == 1) {
    const Box Bf = seg_box_d(a.gf, q);
    for (int d = 0; d < 3; ++d) {
      flo[d] = Bf.a[d] / 2;
      fhi[d] = Bf.b[d] / 2;
    }
  }
  Walk3 wp(threadIdx.x, NT, px, cy);
#pragma unroll
  for (int t = 0; t < kBoxSlots; ++t) {
    const int s = threadIdx.x + t * NT;
    const int xp = wp.i, yy = wp.j, zz = wp.k;
    wp.next();
    li[t] = 0;
    gi[t] = 0;
    fl[t] = 0;
    r0[t] = r1[t] = 0;
    if (s < np) {
      const int x = B.a[0] + 2 * xp, y = B.a[1] + yy, z = B.a[2] + zz;
      li[t] = ((z - B.o[2]) * m + (y - B.o[1])) * m + (x - B.o[0]);
      gi[t] = ((z - Br.o[2]) * a.gr.m + (y - Br.o[1])) * a.gr.m + (x - Br.o[0]);
      const bool two = x + 1 < B.b[0];
      const int byz = (y == 0) + (y == n - 1) + (z == 0) + (z == n - 1);
      const unsigned nb0 = byz + (x == 0) + (x == n - 1), nb1 = byz + (x + 1 == n - 1);
      const bool fyz = y >= flo[1] && y < fhi[1] && z >= flo[2] && z < fhi[2];
      const bool f0 = fyz && x >= flo[0] && x < fhi[0];
      const bool f1 = fyz && x + 1 >= flo[0] && x + 1 < fhi[0];
      fl[t] = ((x + y + z) & 1) | (two ? 2u : 0u) | (nb0 << 2) | (nb1 << 4) | (f0 ? 64u : 0u) |
              (f1 ? 128u : 0u);
      r0[t] = rb[gi[t]];
      if (two) r1[t] = rb[gi[t] + 1];
      ns = t + 1;
    }
  }
  // load the box (u, or u + P(d)) in batches of LB cells per thread, every
  // load of a batch in flight together (lanes outside the domain read element
  // 0 and store 0)
  constexpr int LB = PRO == PRO_LOAD ? kBoxLoads : kBoxLoadsCorrect;
  if (dma) {
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // the copy has landed in LDS
    __syncthreads();
    // zero the box's slabs outside the domain (boundary segments)
    for (int d = 0; d < 3; ++d) {
      const int wl = B.o[d] < 0 ? -B.o[d] : 0, wh = B.o[d] + m > n ? B.o[d] + m - n : 0;
      for (int side = 0; side < 2; ++side) {
        const int w = side ? wh : wl, s0 = side ? m - wh : 0;
        const int cnt = w * m2;
        for (int c = threadIdx.x; c < cnt; c += NT) {
          const int cz = udiv_small(c, m2), r = c - cz * m2, j = udiv_small(r, m), i = r - j * m;
          const int k = s0 + cz;
          // k runs along dimension d, (i, j) over the other two
          const int l = d == 0 ? (j * m + i) * m + k : d == 1 ? (j * m + k) * m + i : (k * m + j) * m + i;
          bu[l] = (T)0;
        }
      }
    }
  }
  Walk3 wl(threadIdx.x, NT, m, m);
  for (int base = dma ? mc : 0; base < mc; base += LB * NT) {
    T vu[LB], vd[LB], vt[LB];
    unsigned vin = 0;
#pragma unroll
    for (int r = 0; r < LB; ++r) {
      const int c = base + threadIdx.x + r * NT;
      const int x = B.o[0] + wl.i, y = B.o[1] + wl.j, z = B.o[2] + wl.k;
      wl.next();
      const bool in = c < mc && in_dom(n, x, y, z);
      vin |= (in ? 1u : 0u) << r;
      vu[r] = ub[in ? c : 0];
      if (PRO == PRO_CORRECT) {
        const long long ic = in ? at(a.gc, Bc, x >> 1, y >> 1, z >> 1) : 0;
        vd[r] = a.d[ic];
        vt[r] = a.dt[ic];
      }
    }
#pragma unroll
    for (int r = 0; r < LB; ++r) {
      const T v = PRO == PRO_CORRECT ? vu[r] + (vd[r] - vt[r]) : vu[r];
      vu[r] = ((vin >> r) & 1u) ? v : (T)0;
      const int c = base + threadIdx.x + r * NT;
      if (c < mc) bu[c] = vu[r];
    }

  }

  __syncthreads();

  // FAS prologue: t = the loaded box, where the finer level's correction reads
  // it (the parents of the finer segment's stored cells, inside the domain)
  if (fas) {
    const Box Bf = seg_box_d(a.gf, q);
    int tlo[3], tw[3];
    for (int d = 0; d < 3; ++d) {
      int lo = Bf.o[d] >> 1, hi = (Bf.o[d] + a.gf.m - 1) >> 1;
      lo = max(max(lo, B.o[d]), 0);
      hi = min(min(hi, B.o[d] + m - 1), n - 1);
      tlo[d] = lo - B.o[d];
      tw[d] = hi - lo + 1;
    }
    const int tc = tw[0] * tw[1] * tw[2];
    Walk3 wt(threadIdx.x, NT, tw[0], tw[1], tc);
    for (int c = threadIdx.x; c < tc; c += NT, wt.next()) {
      const int l = ((tlo[2] + wt.k) * m + (tlo[1] + wt.j)) * m + (tlo[0] + wt.i);
      a.t[B.base + l] = bu[l];
    }
  }

  const double s2 = (double)n * (double)n;
  // L u of the cell at LDS index l with nb boundary faces (Eq. 2, in FP64)
  auto lap = [&](int l, unsigned nb) -> double {
    const double s = (((double)bu[l - 1] + (double)bu[l + 1]) +
                      ((double)bu[l - m] + (double)bu[l + m])) +
                     ((double)bu[l - m2] + (double)bu[l + m2]);
    return (s - (double)(6 + nb) * (double)bu[l]) * s2;
  };

  if (fas) {  // rhs = (R res on F, else 0) + L u, kept in registers and stored
#pragma unroll
    for (int t = 0; t < kBoxSlots; ++t) {
      if (t < ns) {
        unsigned f = fl[t];
        asm volatile("" : "+v"(f));
        const double l0 = lap(li[t], (f >> 2) & 3u);
        r0[t] = (T)(((f & 64u) ? (double)r0[t] : 0.0) + l0);
        a.rhsw[Br.base + gi[t]] = r0[t];
        if (f & 2u) {
          const double l1 = lap(li[t] + 1, (f >> 4) & 3u);
          r1[t] = (T)(((f & 128u) ? (double)r1[t] : 0.0) + l1);
          a.rhsw[Br.base + gi[t] + 1] = r1[t];
        }
      }
    }
  }

  if (fas) __syncthreads();  // the prologue read u before the sweeps write it

  // red-black sweeps: per group of slots, all loads, then the stores (cells
  // of one colour read only the other colour).  The slot flags pass through
  // an empty asm so that the per-colour selections are formed in the sweep
  // instead of being hoisted for both colours (which exhausts registers).
  constexpr int G = 8;  // slots per group: bounds the loads in flight
  const T h2 = a.h2;
  for (int it = 0; it < a.nu; ++it)
    for (int col = 0; col < 2; ++col) {
#pragma unroll
      for (int g0 = 0; g0 < kBoxSlots; g0 += G) {
        T nv[G];
        int lw[G];
#pragma unroll
        for (int t = g0; t < g0 + G; ++t) {
          nv[t - g0] = 0;
          lw[t - g0] = -1;
          if (t < ns) {
            unsigned f = fl[t] ^ (unsigned)col;
            asm volatile("" : "+v"(f));
            const int off = f & 1;  // which cell of the pair has colour col
            const int l = li[t] + off;
            const T s = ((bu[l - 1] + bu[l + 1]) + (bu[l - m] + bu[l + m])) + (bu[l - m2] + bu[l + m2]);
            nv[t - g0] = (s - h2 * (off ? r1[t] : r0[t])) * box_inv_diag<T>((f >> (off ? 4 : 2)) & 3u);
            if (!off || (f & 2u)) lw[t - g0] = l;
          }
        }
#pragma unroll
        for (int t = 0; t < G; ++t)
          if (lw[t] >= 0) bu[lw[t]] = nv[t];
      }
      __syncthreads();
    }

  // residuals of the own cells (kept over the right-hand side registers)
  const bool epi = PRO == PRO_LOAD && a.rmode >= 0;
  if (epi) {
#pragma unroll
    for (int t = 0; t < kBoxSlots; ++t) {
      if (t < ns) {
        unsigned f = fl[t];
        asm volatile("" : "+v"(f));
        r0[t] = (T)((double)r0[t] - lap(li[t], (f >> 2) & 3u));
        if (f & 2u) r1[t] = (T)((double)r1[t] - lap(li[t] + 1, (f >> 4) & 3u));
      }
    }
  }

  // write back: the compute region, and the ghosts when the prologue changed them
  if constexpr (PRO == PRO_CORRECT) {
    Walk3 ww(threadIdx.x, NT, m, m);
    for (int c = threadIdx.x; c < mc; c += NT, ww.next()) {
      const int x = B.o[0] + ww.i, y = B.o[1] + ww.j, z = B.o[2] + ww.k;
      if (in_dom(n, x, y, z)) ub[c] = bu[c];
    }
  } else {  // only C (inside the domain): walk C itself
    const int cc = cx * cy * cz;
    Walk3 ww(threadIdx.x, NT, cx, cy, cc);
    for (int c = threadIdx.x; c < cc; c += NT, ww.next()) {
      const int l = ((B.a[2] - B.o[2] + ww.k) * m + (B.a[1] - B.o[1] + ww.j)) * m + (B.a[0] - B.o[0] + ww.i);
      ub[l] = bu[l];
    }
  }
  if (!epi) return;

  // epilogue: restriction of u, then of the residuals (written over u in LDS)
  int lo[3], hi[3];
  if (a.rmode == 0) {
    for (int d = 0; d < 3; ++d) {
      lo[d] = B.a[d] / 2;
      hi[d] = B.b[d] / 2;
    }
  } else {
    const int S = gu.S, e = udiv_small(a.gcr.n, S);
    const int qy = udiv_small(q, S), qz = udiv_small(qy, S);
    const int p[3] = {q - qy * S, qy - qz * S, qz};
    for (int d = 0; d < 3; ++d) {
      lo[d] = p[d] * e;
      hi[d] = (p[d] + 1) * e;
    }
  }
  const Box Bo = seg_box_d(a.gcr, q);
  const int ex = hi[0] - lo[0], ey = hi[1] - lo[1], ncc = ex * ey * (hi[2] - lo[2]);
  auto child0 = [&](const Walk3& w, long long& id) -> int {  // LDS index of the (0,0,0) child
    const int I = w.i, J = w.j, K = w.k;
    id = at(a.gcr, Bo, lo[0] + I, lo[1] + J, lo[2] + K);
    return ((2 * (lo[2] + K) - B.o[2]) * m + (2 * (lo[1] + J) - B.o[1])) * m +
           (2 * (lo[0] + I) - B.o[0]);
  };
  auto sum8 = [&](int l) -> double {
    return ((((double)bu[l] + (double)bu[l + 1]) + ((double)bu[l + m] + (double)bu[l + m + 1])) +
            (((double)bu[l + m2] + (double)bu[l + m2 + 1]) +
             ((double)bu[l + m2 + m] + (double)bu[l + m2 + m + 1])));
  };
  Walk3 wu(threadIdx.x, NT, ex, ey);
  for (int cc = threadIdx.x; cc < ncc; cc += NT, wu.next()) {
    long long id;
    const int l = child0(wu, id);
    a.uc[id] = (T)(sum8(l) / 8.0);
  }
  __syncthreads();
#pragma unroll
  for (int t = 0; t < kBoxSlots; ++t) {
    if (t < ns) {
      bu[li[t]] = r0[t];
      if (fl[t] & 2u) bu[li[t] + 1] = r1[t];
    }
  }
  __syncthreads();
  Walk3 wr(threadIdx.x, NT, ex, ey);
  for (int cc = threadIdx.x; cc < ncc; cc += NT, wr.next()) {
    long long id;
    const int l = child0(wr, id);
    a.rc[id] = (T)(sum8(l) / 8.0);
  }
}

}  // namespace fmg
