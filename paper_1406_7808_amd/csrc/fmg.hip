// fmg.hip -- plan, schedule and C interface of the solver (include/fmg.h).
//
// The schedule follows the paper (arXiv:1406.7808):
//   FMG (Fig. 2): u_0 = L_0^-1 f_0; for l = 1..M: u_l = Pi u_{l-1},
//     S^alpha, one FAS V-cycle (Fig. 1) with rhs f_l;
//   SR-FMG (Fig. 5): the same up to the transition level T, then for each
//     SR stage l = T+1..M every segment interpolates onto its compute region
//     and GSR ghosts, smooths, and runs the SR V-cycle (Fig. 6), whose only
//     cross-segment step is the owner-computes restriction to level T and the
//     global V-cycle there;
//   mixed precision: u = FMG32(f); repeat: r = f - L u in FP64, u += FMG32(r).
// All kernels of one solve are enqueued on the caller's stream; the host never
// waits inside a solve.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <set>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/fmg.h"
#include "grid.hpp"
#include "kernels_coarse.hpp"
#include "kernels_cols.hpp"
#include "kernels_descend.hpp"
#include "kernels_fused.hpp"
#include "kernels_norms.hpp"
#include "kernels_simple.hpp"

using namespace fmg;

// ---------------------------------------------------------------------------
// errors

static thread_local std::string g_err;

static int32_t fail(int32_t st, const std::string& msg) {
  g_err = msg;
  return st;
}

struct hip_error : std::runtime_error {
  using std::runtime_error::runtime_error;
};

static void hipcheck(hipError_t e, const char* what) {
  if (e != hipSuccess) throw hip_error(std::string(what) + ": " + hipGetErrorString(e));
}


// ---------------------------------------------------------------------------
// parameter validation (host only)

static const int kMaxSweeps = 8;
static const int kMaxCoarse = 8;

static std::string check(int32_t N, const fmg_params* p) {
  char buf[256];
  if (!p) return "params is NULL";
  if (N < 1) return "N must be >= 1";
  if (N > 2048) return "N must be <= 2048";
  int L = p->levels;
  if (L < 1 || L > 12) return "levels must be in [1, 12]";
  int n0 = N >> (L - 1);
  if ((n0 << (L - 1)) != N || n0 < 1) {
    snprintf(buf, sizeof buf, "N=%d is not n0 * 2^(levels-1) for levels=%d", N, L);
    return buf;
  }
  if (n0 > kMaxCoarse) {
    snprintf(buf, sizeof buf, "coarsest edge %d exceeds %d (add levels)", n0, kMaxCoarse);
    return buf;
  }
  int K = p->sr_levels, S = p->segments_per_dim;
  if (K < 0 || K > L - 1) return "sr_levels must be in [0, levels-1]";
  if (S < 1 || S > 40) return "segments_per_dim must be in [1, 40]";
  if (p->nu_pre < 0 || p->nu_pre > kMaxSweeps || p->nu_post < 0 || p->nu_post > kMaxSweeps ||
      p->alpha < 0 || p->alpha > kMaxSweeps)
    return "nu_pre, nu_post and alpha must be in [0, 8]";
  if (p->precision != FMG_FP64 && p->precision != FMG_FP32_REFINED) return "unknown precision";
  if (p->refine_iters < 0 || p->refine_iters > 8) return "refine_iters must be in [0, 8]";
  if (K > 0) {
    if (N % (S << K) != 0) {
      snprintf(buf, sizeof buf,
               "N=%d not divisible by segments_per_dim << sr_levels = %d (each segment must own "
               "a transition-level cell)",
               N, S << K);
      return buf;
    }
    if (!p->buffer_schedule) return "buffer_schedule is NULL with sr_levels > 0";
    for (int i = 0; i < K; ++i) {
      int J = p->buffer_schedule[i];
      if (J < 0 || (J & 1)) {
        snprintf(buf, sizeof buf, "buffer_schedule[%d]=%d must be even and >= 0", i, J);
        return buf;
      }
      if (J > N) return "buffer width larger than the grid";
      if (i + 1 < K && 2 * p->buffer_schedule[i + 1] < J) {
        snprintf(buf, sizeof buf,
                 "buffer_schedule[%d]=%d must be >= half of buffer_schedule[%d]=%d", i + 1,
                 p->buffer_schedule[i + 1], i, J);
        return buf;
      }
    }
  }
  return "";
}

// ---------------------------------------------------------------------------
// coarsest-level inverse (host, FP64): A e_c by the 7-point rule with
// boundary ghosts -u_c, then Gauss-Jordan with partial pivoting.

static bool coarse_inverse(int n, std::vector<double>& inv) {
  int mm = n * n * n;
  std::vector<double> A((size_t)mm * mm, 0.0);
  double h2i = (double)n * n;
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        int r = (k * n + j) * n + i;
        int nb = 0;
        const int d[6][3] = {{-1, 0, 0}, {1, 0, 0}, {0, -1, 0}, {0, 1, 0}, {0, 0, -1}, {0, 0, 1}};
        for (auto& e : d) {
          int a = i + e[0], b = j + e[1], c = k + e[2];
          if (in_dom(n, a, b, c))
            A[(size_t)r * mm + (c * n + b) * n + a] += h2i;
          else
            ++nb;
        }
        A[(size_t)r * mm + r] -= (6 + nb) * h2i;
      }
  inv.assign((size_t)mm * mm, 0.0);
  for (int r = 0; r < mm; ++r) inv[(size_t)r * mm + r] = 1.0;
  for (int c = 0; c < mm; ++c) {
    int piv = c;
    for (int r = c + 1; r < mm; ++r)
      if (std::fabs(A[(size_t)r * mm + c]) > std::fabs(A[(size_t)piv * mm + c])) piv = r;
    if (A[(size_t)piv * mm + c] == 0.0) return false;
    if (piv != c)
      for (int t = 0; t < mm; ++t) {
        std::swap(A[(size_t)c * mm + t], A[(size_t)piv * mm + t]);
        std::swap(inv[(size_t)c * mm + t], inv[(size_t)piv * mm + t]);
      }
    double d = 1.0 / A[(size_t)c * mm + c];
    for (int t = 0; t < mm; ++t) {
      A[(size_t)c * mm + t] *= d;
      inv[(size_t)c * mm + t] *= d;
    }
    for (int r = 0; r < mm; ++r) {
      if (r == c) continue;
      double l = A[(size_t)r * mm + c];
      if (l == 0.0) continue;
      for (int t = 0; t < mm; ++t) {
        A[(size_t)r * mm + t] -= l * A[(size_t)c * mm + t];
        inv[(size_t)r * mm + t] -= l * inv[(size_t)c * mm + t];
      }
    }
  }
  return true;
}

// ---------------------------------------------------------------------------
// plan

template <class T>
struct Hier {
  std::vector<Geo> geo;          // storage geometry of u, t, rhs on each level
  std::vector<T*> u, t, rhs, f;  // f[l]: global right-hand-side hierarchy
  // the FAS right-hand side a column-smoother pass forms on a small global
  // level (a separate array: the pass's overlapping tiles still read rhs)
  std::vector<T*> rf;
  // The temporally blocked smoother reads one copy of u and writes the other
  // (tiles overlap by their halo, so an in-place update would race); u[l] is
  // the current copy, ua[l] / ub[l] the pair.
  std::vector<T*> ua, ub;
};

// Per-launch timing: when enabled, every launch of a solve is bracketed by two
// HIP events on the solve's stream and tagged with its kernel name and the
// algorithmic bytes it must move (the unique cells it reads and writes).
struct Prof {
  struct Rec {
    const char* name;
    int level;  // -1: not tied to one level
    hipEvent_t a, b;
    double bytes;
  };
  bool on = false;
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e;
    hipcheck(hipEventCreate(&e), "hipEventCreate");
    return e;
  }
  void recycle() {
    for (auto& r : recs) {
      pool.push_back(r.a);
      pool.push_back(r.b);
    }
    recs.clear();
  }
  ~Prof() {
    recycle();
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

struct fmg_plan {
  int N = 0, L = 0, K = 0, T = 0, S = 1, n0 = 1, device = 0;
  int nu1 = 2, nu2 = 2, alpha = 1, precision = FMG_FP64, refine = 2;
  bool fused = true;          // temporally blocked smoother (else single-cell kernels)
  bool zres = true;           // large global levels: the last pre-smoothing pass of two
                              // half-sweeps also restricts (residual epilogue)
  int Lc = 0;                 // global levels 0..Lc run in the persistent coarse kernel
  int lds_max = 0;            // LDS bytes a workgroup may use (box-resident smoother)
  int max_stages = 4;         // half-sweeps per temporally blocked launch (2 or 4)
  bool seg_inplace = true;    // segment levels: in place, one workgroup per segment
  bool use_box = true;        // segment levels whose box fits LDS: box-resident smoother
  std::set<const void*> lds_attr;  // kernels already allowed the whole LDS
  std::vector<double*> ck;         // level checkpoints (empty: none)
  long long target_blocks = 0;  // workgroups a fused launch aims for (0: chosen per pass)
  int tile_x = 0;               // tile width of the passes over two copies (0: cost model)
  int ncu = 256;                // compute units of the device
  int nxcd = 8;               // L2 domains (XCDs) the blocks are dealt to
  std::vector<int> J;  // J[l] for SR levels, indexed by level
  Hier<double> h64;
  Hier<float> h32;
  double* Ainv = nullptr;
  double* ws_finest = nullptr;  // second copy of the finest global FP64 level
  bool finest_odd = false;      // the finest level ends in its second copy
  float* r32 = nullptr;  // FP32 right-hand side of the inner solves
  double* vpart = nullptr;  // norm partials of the V-cycle iteration (global FP64 plans)
  Prof prof;
  bool virt = false;              // workspace is virtual (schedule model only)
  uintptr_t virt_next = 1 << 20;  // next virtual address
  long long model_launches = 0;   // launches walked by a dry run
  double model_bytes = 0;         // their algorithmic bytes
  std::vector<void*> allocs;
  std::vector<size_t> sizes;
  long long bytes = 0;
};

static void* dalloc(fmg_plan* P, size_t bytes) {
  void* p = nullptr;
  if (bytes == 0) return nullptr;
  if (P->virt) {  // schedule model: distinct non-null addresses, no device memory
    p = (void*)P->virt_next;
    P->virt_next += (bytes + 255) / 256 * 256;
    P->bytes += (long long)bytes;
    return p;
  }
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    throw std::bad_alloc();
  }
  P->allocs.push_back(p);
  P->sizes.push_back(bytes);
  P->bytes += (long long)bytes;
  return p;
}

static long long cube(long long x) { return x * x * x; }

// Two-copy passes on levels of edge up to kLatencyEdge are chains of memory
// round trips rather than streams.  On global levels they run in the column
// smoother, which loads a whole z chunk at once; on segment levels (reached
// only with the box and in-place smoothers off) the z march takes one column
// per thread and keeps two planes in flight, so a step's loads have two steps
// to arrive (four in flight were slower)
constexpr int kLatencyEdge = 64;

template <class T>
static void build_hier(fmg_plan* P, Hier<T>& H, bool finest_external) {
  int L = P->L;
  H.geo.resize(L);
  H.u.assign(L, nullptr);
  H.ua.assign(L, nullptr);
  H.ub.assign(L, nullptr);
  H.t.assign(L, nullptr);
  H.rhs.assign(L, nullptr);
  H.rf.assign(L, nullptr);
  H.f.assign(L, nullptr);
  for (int l = 0; l < L; ++l) {
    int n = P->N >> (L - 1 - l);
    bool sr = l > P->T;
    H.geo[l] = sr ? segment_geo(n, P->S, P->J[l]) : global_geo(n);
    long long cnt = sr ? cube(P->S) * H.geo[l].sstride : cube(n);
    if (l < L - 1) H.f[l] = (T*)dalloc(P, sizeof(T) * cube(n));
    // the caller's array is one copy of the finest global level
    if (!(l == L - 1 && !sr && finest_external)) H.ua[l] = (T*)dalloc(P, sizeof(T) * cnt);
    if (l > 0) H.ub[l] = (T*)dalloc(P, sizeof(T) * cnt);
    H.u[l] = H.ua[l];
    if (l < L - 1) {
      H.t[l] = (T*)dalloc(P, sizeof(T) * cnt);
      H.rhs[l] = (T*)dalloc(P, sizeof(T) * cnt);
      if (!sr) H.rf[l] = (T*)dalloc(P, sizeof(T) * cnt);  // FAS right-hand side (global levels)
    }
  }
}

// ---------------------------------------------------------------------------
// schedule

static const int kBlock = 256;

static dim3 grid_for(long long cells, int nseg) {
  return dim3((unsigned)((cells + kBlock - 1) / kBlock), (unsigned)nseg);
}

// planes in flight per thread in the temporally blocked smoother: one plane,
// whose loads overlap the half-sweeps of a whole step (deeper rings make the
// register allocator copy in-flight registers at the loop back edge)
template <int NS>
constexpr int kPrefetch = 1;


template <class X>
static bool nonnull(const X&) { return true; }
template <class X>
static bool nonnull(X* p) { return p != nullptr; }
static bool geo_ok(const Geo& g) { return g.n >= 1 && g.m >= 1 && g.S >= 1 && g.g >= 1; }
template <class X>
static bool nonnull(const SmoothArgs<X>& a) {
  return a.uin && a.u && a.rhs && (a.uin != a.u || a.inplace) && geo_ok(a.gu) && geo_ok(a.gr) &&
         geo_ok(a.gc) && (a.rmode < 0 || (a.uc && a.rc && geo_ok(a.gcr) && a.rmode <= 1)) &&
         a.txw > 2 && a.tyw > 2 && a.ntx >= 1 && a.nty >= 1 && a.ntz >= 1 && a.zc >= 1 &&
         a.nxcd >= 1;
}
template <class X>
static bool nonnull(const DescArgs<X>& a) {
  return a.u && a.rhs && a.uc && a.rc && geo_ok(a.gu) && geo_ok(a.gr) && geo_ok(a.gc) &&
         a.ctx >= 1 && a.cty >= 1 && (2 * a.ctx + 2) * (2 * a.cty + 2) <= kDescThreads &&
         a.kc >= 1 && a.ntx >= 1 && a.nty >= 1 && a.ntz >= 1 && a.nxcd >= 1 &&
         (a.mode == 0 || a.mode == 1);
}
template <class X>
static bool nonnull(const BoxArgs<X>& a) {
  return a.u && a.rhs && a.d && a.dt && geo_ok(a.gu) && geo_ok(a.gr) && geo_ok(a.gc) &&
         (!a.fas || (a.rhsw && a.t && geo_ok(a.gf))) &&
         (a.rmode < 0 || (a.uc && a.rc && geo_ok(a.gcr) && a.rmode <= 1));
}
template <class X>
static bool nonnull(const CoarseArgs<X>& a) {
  if (!a.Ainv || !a.u[0] || (a.mode == 1 && !a.rt)) return false;
  for (int l = 0; l <= a.top; ++l) {
    if (!a.u[l] || (a.mode == 0 && !a.f[l])) return false;
    if (l < a.top && (!a.t[l] || !a.r[l])) return false;
  }
  return true;
}

// profile label of one k_smooth_z instantiation, e.g. "k_smooth_z<load,ns2,ry1>"
template <int NS, int PRO, int RY, int RES, int PF, int FAS>
static const char* zlabel() {
  static const std::string s = std::string("k_smooth_z<") +
                               (PRO == PRO_CORRECT ? "correct" : PRO == PRO_INTERP ? "interp" : "load") +
                               ",ns" +
                               std::to_string(NS) + ",ry" + std::to_string(RY) +
                               (RES ? ",res" : "") + (FAS ? ",fas" : "") +
                               (PF > 1 ? ",pf" + std::to_string(PF) : "") + ">";
  return s.c_str();
}

// profile label of one k_smooth_cols instantiation, e.g. "k_smooth_cols<load,ns4,res>"
template <int NS, int PRO, int RES>
static const char* clabel() {
  static const std::string s = std::string("k_smooth_cols<") +
                               (PRO == PRO_CORRECT ? "correct" : PRO == PRO_INTERP ? "interp" : "load") +
                               ",ns" + std::to_string(NS) + (RES ? ",res" : "") + ">";
  return s.c_str();
}

template <class T>
struct Exec {
  using A = T;  // smoothing arithmetic: FP64 or FP32
  fmg_plan* P;
  Hier<T>& H;
  hipStream_t s;
  bool dry = false;  // walk the schedule without launching (buffer bookkeeping)
  int lvl = -1;      // level of the launches being issued (profile label)
  // the solve's final pass may write the genuine cells to fin_out (added when
  // fin_acc) itself; fin_done records that it did
  // level checkpoints are taken by FP64 solves when the caller set them
  bool checkpoints() const { return sizeof(T) == 8 && !P->ck.empty(); }

  // level l's solution after its FMG stage into its checkpoint (global
  // levels: a copy; segment levels: the genuine cells)
  void checkpoint(int l) {
    if (!checkpoints() || !P->ck[l]) return;
    const Geo& G = H.geo[l];
    lvl = l;
    if (!G.ghost) {
      if (!dry)
        hipcheck(hipMemcpyAsync(P->ck[l], H.u[l], sizeof(T) * (size_t)cube(G.n),
                                hipMemcpyDeviceToDevice, s),
                 "hipMemcpyAsync");
      return;
    }
    run("k_gather", (sizeof(T) + 8.0) * cube(G.n), grid_for(cube(G.g), nseg(l)), dim3(kBlock),
        k_gather<T>, P->ck[l], (const T*)H.u[l], G, 0);
  }

  double* want_out = nullptr;  // where this solve's genuine cells go (K > 0)
  int want_acc = 0;
  double* fin_out = nullptr;
  int fin_acc = 0;
  bool fin_done = false;

  int nseg(int l) const { return l > P->T ? P->S * P->S * P->S : 1; }

  template <class K, class... Args>
  void run(const char* name, double bytes, dim3 grid, dim3 block, K kern, Args... args) {
    run_shm(name, bytes, grid, block, 0, kern, args...);
  }

  template <class K, class... Args>
  void run_shm(const char* name, double bytes, dim3 grid, dim3 block, size_t shm, K kern,
               Args... args) {
    if (!(nonnull(args) && ...)) throw hip_error(std::string("internal: invalid launch arguments for ") + name);
    if (grid.x == 0 || grid.y == 0) throw hip_error(std::string("internal: empty grid for ") + name);
    if (dry) {
      P->model_launches += 1;
      P->model_bytes += bytes;
      return;
    }
    Prof& pr = P->prof;
    hipEvent_t a = nullptr;
    if (pr.on) {
      a = pr.get();
      hipcheck(hipEventRecord(a, s), "hipEventRecord");
    }
    hipLaunchKernelGGL(kern, grid, block, shm, s, args...);
    hipcheck(hipGetLastError(), name);
    if (pr.on) {
      hipEvent_t b = pr.get();
      hipcheck(hipEventRecord(b, s), "hipEventRecord");
      pr.recs.push_back({name, lvl, a, b, bytes});
    }
  }
  int cext(int l) const {  // maximal compute-region edge
    const Geo& G = H.geo[l];
    return (G.g + 2 * G.J) < G.n ? (G.g + 2 * G.J) : G.n;
  }

  // cells summed over all segments of a level: compute regions, and stored
  // cells inside the domain (compute regions plus GSR ghosts)
  static double span_sum(const Geo& G, int grow) {
    double t = 0;
    for (int p = 0; p < G.S; ++p) {
      int a = p * G.g - G.J - grow, b = (p + 1) * G.g + G.J + grow;
      t += (b > G.n ? G.n : b) - (a < 0 ? 0 : a);
    }
    return t;
  }
  static double c_cells(const Geo& G) { double t = span_sum(G, 0); return t * t * t; }
  static double st_cells(const Geo& G) { double t = span_sum(G, G.ghost); return t * t * t; }

  // nu red-black sweeps on level l with the single-cell kernel
  void smooth_simple(int l, const T* rhs, Geo gr, int nu) {
    const Geo& G = H.geo[l];
    double h = 1.0 / (double)G.n;
    A h2 = (A)(h * h);
    int ce = cext(l);
    // per half-sweep: read rhs and the other colour, write this colour
    double bytes = 1.5 * sizeof(T) * c_cells(G);
    for (int it = 0; it < nu; ++it)
      for (int col = 0; col < 2; ++col)
        run("k_gs_half", bytes, grid_for(cube(ce), nseg(l)), dim3(kBlock), k_gs_half<T, A>,
            H.u[l], G, rhs, gr, col, h2, ce);
  }

  // one temporally blocked launch of NS half-sweeps with prologue PRO; RY
  // columns per thread; inpl: one workgroup per segment, updated in place;
  // FAS: a load pass over two copies on a global level first forms the FAS
  // right-hand side rhs + L u, into rf, and t = u
  template <int NS, int RY, int PRO, int RES = 0, int PF = kPrefetch<NS>, int FAS = 0>
  void smooth_z(int l, const T* rhs, Geo gr, const T* c, const T* ct, Geo gc, bool inpl,
                double* out = nullptr, int outmode = 0, int rmode = -1) {
    constexpr int NT = 1024, NC = NT * RY;
    // two workgroups per CU (at most 64 VGPRs) where the kernel fits them
    // (not the latency variant: its launches are small)
    constexpr int WPE =
        (PF == 1 && NS <= 2 && !RES && (RY == 1 || (sizeof(T) == 4 && PRO == PRO_LOAD && !FAS)))
            ? 8
            : 4;
    const Geo& G = H.geo[l];
    if (PRO != PRO_LOAD && (!c || !ct)) throw hip_error("internal: null coarse increment");
    SmoothArgs<T> a{};
    a.uin = H.u[l];
    a.u = inpl ? H.u[l] : (H.u[l] == H.ua[l] ? H.ub[l] : H.ua[l]);
    a.gu = G;
    H.u[l] = a.u;  // the written copy becomes current
    a.rhs = rhs;
    a.gr = gr;
    a.c = c;
    a.ct = ct;
    a.gc = gc;
    a.inplace = inpl ? 1 : 0;
    if (outmode && (!inpl || !out)) throw hip_error("internal: output epilogue needs an in-place pass");
    a.out = out;
    a.outmode = outmode;
    if (RES != (rmode >= 0) || (RES && (l < 1 || (!inpl && (nseg(l) != 1 || rmode != 0)))))
      throw hip_error("internal: residual epilogue needs an in-place pass or a global level");
    a.rmode = rmode;
    a.uc = RES ? H.u[l - 1] : nullptr;
    a.rc = RES ? H.rhs[l - 1] : nullptr;
    a.gcr = H.geo[l > 0 ? l - 1 : 0];
    if (FAS && (inpl || G.ghost || nseg(l) != 1 || gr.ghost || gr.n != G.n || !H.rf[l] ||
                !H.t[l] || rhs == H.rf[l]))
      throw hip_error("internal: FAS prologue needs a global level over two copies, t and rf");
    a.fas = FAS;
    a.rhsw = FAS ? H.rf[l] : nullptr;
    a.tw = FAS ? H.t[l] : nullptr;
    double h = 1.0 / (double)G.n;
    a.h2 = (T)(h * h);
    int ns = nseg(l);
    if (inpl) {
      // one tile covering the largest compute region plus the halo, one chunk
      const int ce = cext(l);
      if (!G.ghost || (ce + 2 * NS) * (ce + 2 * NS) > NC)
        throw hip_error("internal: segment does not fit one in-place tile");
      a.txw = a.tyw = ce + 2 * NS;
      a.ntx = a.nty = a.ntz = 1;
      a.zc = ce;
    } else {
      // every stored cell inside the domain is written, so the new copy is whole
      int wext = cext(l) + 2 * G.ghost;
      if (wext > G.n) wext = G.n;
      // tile halo (one more for a residual epilogue, whose restriction also
      // needs even output extents: coarse cells are not split between tiles)
      constexpr int HH = NS + RES;
      // tile shape: the fewest loaded columns covering the write region, or
      // the tuned width (clamped to what the pass admits)
      long long best = -1;
      // even widths: the kernel deals each row's columns to two colour classes
      auto search = [&](int tlo, int thi) {
        for (int tx = tlo; tx <= thi && tx * (2 * HH + 2) <= NC; tx += 2) {
          int ty = NC / tx;
          if (ty > wext + 2 * HH) ty = wext + 2 * HH;
          if (RES) ty &= ~1;
          if (ty < 2 * HH + 2) continue;
          long long cost = (long long)((wext + tx - 2 * HH - 1) / (tx - 2 * HH)) *
                           ((wext + ty - 2 * HH - 1) / (ty - 2 * HH)) * tx * ty;
          if (tx < 16) cost += cost / 4;  // short rows load poorly
          if (best < 0 || cost < best) {
            best = cost;
            a.txw = tx;
            a.tyw = ty;
          }
        }
      };
      if (P->tile_x) {
        const int tx = std::max(2 * HH + 2, std::min(P->tile_x, NC / (2 * HH + 2)) & ~1);
        search(tx, tx);
      }
      if (best < 0) search(2 * HH + 2, 256);
      if (best < 0) throw hip_error("internal: no tile shape fits the pass");
      const int SX = a.txw - 2 * HH, SY = a.tyw - 2 * HH;
      a.ntx = (wext + SX - 1) / SX;
      a.nty = (wext + SY - 1) / SY;
      long long bxy = (long long)a.ntx * a.nty * ns;
      // large levels keep chunks at least 2 NS deep (recomputed halo planes);
      // small, L2-resident levels split finely to shorten the serial z march
      int zmax = wext <= 64 ? (wext + 1) / 2 : wext / (2 * NS);
      if (zmax < 1) zmax = 1;
      auto chunk = [&](int nz) {  // planes per chunk for nz chunks
        int zc = (wext + nz - 1) / nz;
        if (RES) zc += zc & 1;  // chunks of whole coarse planes
        return zc;
      };
      int ntz;
      if (P->target_blocks == 0 && wext > 64) {
        // chosen by rounds of resident workgroups: every chunk marches its
        // planes plus NS (+1) halo planes, and a launch takes as many such
        // marches as it has rounds of workgroups, the last one too however
        // few it holds
        const long long slots = (long long)P->ncu * (WPE / 4);
        long long bestc = -1;
        ntz = 1;
        for (int nz = 1; nz <= zmax; ++nz) {
          const int zc = chunk(nz);
          const int nzr = (wext + zc - 1) / zc;
          const long long rounds = (bxy * nzr + slots - 1) / slots;
          const long long c = rounds * (zc + 2 * NS + RES);
          if (bestc < 0 || c < bestc) {  // ties: fewer, longer chunks
            bestc = c;
            ntz = nz;
          }
        }
      } else {
        const long long tb = P->target_blocks ? P->target_blocks : 1024;
        ntz = (int)((tb + bxy - 1) / bxy);
        if (ntz > zmax) ntz = zmax;
        if (ntz < 1) ntz = 1;
      }
      a.zc = chunk(ntz);
      a.ntz = (wext + a.zc - 1) / a.zc;
    }
    if (a.txw & 1) throw hip_error("internal: the smoother's tile width must be even");
    // the interpolation prologue loads the coarse columns under a tile, one per thread
    if (PRO == PRO_INTERP && ((a.txw >> 1) + 3) * ((a.tyw >> 1) + 3) > NT)
      throw hip_error("internal: tile too wide for the interpolation prologue");
    a.nxcd = ns > 1 ? 1 : P->nxcd;
    int nt = a.ntx * a.nty * a.ntz;
    int per = (nt + a.nxcd - 1) / a.nxcd;
    // u read: whole, plus a quarter for the correction's w and t, or only the
    // coarse u (an eighth) for the interpolation prologue
    double rd = PRO == PRO_CORRECT ? 1.25 : PRO == PRO_INTERP ? 0.125 : 1.0;
    double bytes = sizeof(T) * (2.0 + rd) * c_cells(G);
    if (outmode)  // u is not stored; the genuine cells go out in FP64 (read too when added)
      bytes += 8.0 * outmode * cube(P->N) - sizeof(T) * c_cells(G);
    if (RES)  // uc and rc on the coarse target
      bytes += 2.0 * sizeof(T) * (rmode == 0 ? c_cells(G) / 8.0 : cube(H.geo[l - 1].n));
    if (FAS) bytes += 2.0 * sizeof(T) * c_cells(G);  // rhs and t written
    run(zlabel<NS, PRO, RY, RES, PF, FAS>(), bytes,
        dim3(per * a.nxcd, ns), dim3(NT), k_smooth_z<T, NS, PRO, NT, RY, PF, WPE, RES, FAS>,
        a);
  }

  // NS half-sweeps with prologue PRO on a small global level, one column
  // per thread with its whole z chunk in registers (two copies); RES: the
  // pass also restricts u and the residual to level l - 1; fas: it first
  // forms the FAS right-hand side rhs + L u and t = u of this level
  // ZC: output planes per z chunk (each chunk also loads 2 (NS + RES) halo
  // planes)
  template <int NS, int PRO, int RES, int ZC = 2>
  void smooth_cols(int l, const T* rhs, Geo gr, const T* c, const T* ct, Geo gc, int fas = 0) {
    constexpr int NT = 1024, HH = NS + RES;
    const Geo& G = H.geo[l];
    const int n = G.n;
    if (G.ghost || nseg(l) != 1 || (RES && l < 1) || n < 2)
      throw hip_error("internal: the column smoother takes global levels of edge 2 and up");
    if (PRO != PRO_LOAD && (!c || (PRO == PRO_CORRECT && !ct)))
      throw hip_error("internal: null coarse increment");
    if (fas && (PRO != PRO_LOAD || !H.t[l] || !H.rf[l]))
      throw hip_error("internal: FAS prologue without a load pass, t or its rhs array");
    SmoothArgs<T> a{};
    a.uin = H.u[l];
    a.u = H.u[l] == H.ua[l] ? H.ub[l] : H.ua[l];
    a.gu = G;
    H.u[l] = a.u;  // the written copy becomes current
    a.rhs = rhs;
    a.gr = gr;
    a.c = c;
    a.ct = ct;
    a.gc = gc;
    a.inplace = 0;
    a.rmode = RES ? 0 : -1;
    a.uc = RES ? H.u[l - 1] : nullptr;
    a.rc = RES ? H.rhs[l - 1] : nullptr;
    a.gcr = H.geo[l > 0 ? l - 1 : 0];
    a.fas = fas;
    a.rhsw = fas ? H.rf[l] : nullptr;
    a.tw = fas ? H.t[l] : nullptr;
    const double h = 1.0 / (double)n;
    a.h2 = (T)(h * h);
    // tile shape: the fewest loaded columns covering the level; even extents,
    // so that every output region starts on even x and y
    long long best = -1;
    for (int tx = 2 * HH + 2; tx <= 256 && tx * (2 * HH + 2) <= NT; tx += 2) {
      int ty = NT / tx;
      if (ty > n + 2 * HH) ty = n + 2 * HH;
      ty &= ~1;
      if (ty < 2 * HH + 2) continue;
      long long cost = (long long)((n + tx - 2 * HH - 1) / (tx - 2 * HH)) *
                       ((n + ty - 2 * HH - 1) / (ty - 2 * HH)) * tx * ty;
      if (best < 0 || cost < best) {
        best = cost;
        a.txw = tx;
        a.tyw = ty;
      }
    }
    // (the restriction pairs cells: even edges only)
    if (best < 0 || (RES && (n & 1))) throw hip_error("internal: no tile for the column smoother");
    a.ntx = (n + a.txw - 2 * HH - 1) / (a.txw - 2 * HH);
    a.nty = (n + a.tyw - 2 * HH - 1) / (a.tyw - 2 * HH);
    a.ntz = (n + ZC - 1) / ZC;
    a.zc = ZC;
    a.nxcd = P->nxcd;
    const int nt = a.ntx * a.nty * a.ntz;
    const int per = (nt + a.nxcd - 1) / a.nxcd;
    double rd = PRO == PRO_CORRECT ? 1.25 : PRO == PRO_INTERP ? 0.125 : 1.0;
    double bytes = sizeof(T) * (2.0 + rd) * c_cells(G);
    if (RES) bytes += 2.0 * sizeof(T) * c_cells(G) / 8.0;
    if (fas) bytes += 2.0 * sizeof(T) * c_cells(G);  // rhs and t written
    run(clabel<NS, PRO, RES>(), bytes, dim3(per * a.nxcd), dim3(NT),
        k_smooth_cols<T, NS, PRO, RES, ZC>, a);
  }

  template <int PRO>
  void smooth_z_ns(int ns, bool inpl, int l, const T* rhs, Geo gr, const T* c, const T* ct,
                   Geo gc, double* out = nullptr, int outmode = 0, int fas = 0) {
    // one column per thread for FP64 two-stage passes over two copies (few
    // enough registers for two workgroups per CU), else two
    constexpr int RY2 = sizeof(T) == 8 ? 1 : 2;
    if (fas && (inpl || PRO != PRO_LOAD))
      throw hip_error("internal: FAS prologue off a load pass over two copies");
    if (cols_level(l) && !inpl) {
      if (ns == 2) smooth_cols<2, PRO, 0>(l, rhs, gr, c, ct, gc, fas);
      else smooth_cols<4, PRO, 0>(l, rhs, gr, c, ct, gc, fas);
    } else if (fas) {  // a large global level
      if constexpr (PRO == PRO_LOAD) {
        if (ns == 2) smooth_z<2, RY2, PRO_LOAD, 0, kPrefetch<2>, 1>(l, rhs, gr, c, ct, gc, false);
        else smooth_z<4, RY2, PRO_LOAD, 0, kPrefetch<4>, 1>(l, rhs, gr, c, ct, gc, false);
      }
    } else if (!inpl && H.geo[l].n <= kLatencyEdge) {
      if (ns == 2) smooth_z<2, 1, PRO, 0, 2>(l, rhs, gr, c, ct, gc, false);
      else smooth_z<4, 1, PRO, 0, 2>(l, rhs, gr, c, ct, gc, false);
    } else if (ns == 2 && !inpl) smooth_z<2, RY2, PRO>(l, rhs, gr, c, ct, gc, false);
    else if (ns == 2) smooth_z<2, 2, PRO>(l, rhs, gr, c, ct, gc, true, out, outmode);
    else smooth_z<4, 2, PRO>(l, rhs, gr, c, ct, gc, inpl, out, outmode);
  }

  // is level l a small global level, whose fused passes run in the column
  // smoother?
  bool cols_level(int l) const {
    const Geo& G = H.geo[l];
    return !G.ghost && nseg(l) == 1 && G.n <= kLatencyEdge;
  }

  // can the first pre-smoothing pass of level l form its FAS right-hand side
  // (the column smoother's prologue, or the z march's over two copies on a
  // larger global level), so that the restriction into it need not?
  bool pass_fas(int l) const {
    if (!(l > P->Lc && P->fused && P->nu1 > 0)) return false;
    if (cols_level(l)) return true;
    const Geo& G = H.geo[l];
    if (G.ghost || nseg(l) != 1) return false;
    // not when that pass is also the one that restricts (see smooth)
    const int st = 2 * P->nu1, ns = st >= P->max_stages ? P->max_stages : st;
    return !(ns == 2 && st == ns && sizeof(T) == 8 && P->zres);
  }

  // can level l's segments be smoothed in place, one workgroup each, with
  // four half-sweeps per pass?
  bool seg_inplace(int l) const {
    const Geo& G = H.geo[l];
    const int ce = cext(l) + 8;
    return P->seg_inplace && G.ghost && ce * ce <= 2 * 1024;
  }

  // does a segment's whole storage box fit the box-resident smoother?
  bool box_fits(int l) const {
    const Geo& G = H.geo[l];
    if (!G.ghost || !P->use_box) return false;
    long long ce = cext(l);
    long long pairs = (ce + 1) / 2 * ce * ce;
    return cube(G.m) * (long long)sizeof(T) <= P->lds_max && pairs <= kBoxSlots * kBoxThreads;
  }

  // allow a kernel the device's whole LDS per workgroup (once per plan, so
  // once per device)
  void allow_lds(const void* fn, int bytes) {
    if (dry || P->lds_attr.count(fn)) return;
    hipcheck(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, bytes),
             "hipFuncSetAttribute");
    P->lds_attr.insert(fn);
  }

  // fas: form the FAS right-hand side in the prologue (see BoxArgs); rmode >= 0:
  // residual and restriction in the epilogue (0: to F of the coarse segment,
  // 1: owner computes into the global transition level)
  template <int PRO>
  void smooth_box_pro(int l, const T* rhs, Geo gr, int nu, const T* d, const T* dt, Geo gc,
                      int fas, int rmode) {
    const Geo& G = H.geo[l];
    size_t shm = (size_t)cube(G.m) * sizeof(T);
    allow_lds((const void*)k_smooth_box<T, PRO>, P->lds_max);
    BoxArgs<T> a{};
    a.u = H.u[l];
    a.gu = G;
    a.rhs = rhs;
    a.gr = gr;
    a.d = PRO == PRO_CORRECT ? d : H.u[l];
    a.dt = PRO == PRO_CORRECT ? dt : H.u[l];
    a.gc = gc;
    double h = 1.0 / (double)G.n;
    a.h2 = (T)(h * h);
    a.nu = nu;
    a.fas = PRO == PRO_LOAD ? fas : 0;
    a.rhsw = H.rhs[l];
    a.t = H.t[l];
    a.gf = H.geo[l + 1 < P->L ? l + 1 : l];
    a.rmode = PRO == PRO_LOAD ? rmode : -1;
    a.uc = H.u[l - 1];
    a.rc = H.rhs[l - 1];
    a.gcr = H.geo[l - 1];
    if (a.fas && (rhs != H.rhs[l] || l + 1 >= P->L))
      throw hip_error("internal: FAS prologue needs the level's own right-hand side");
    double rd = PRO == PRO_CORRECT ? 1.25 : 1.0;
    double bytes = sizeof(T) * (2.0 + rd) * c_cells(G);
    if (a.fas) {  // rhs written on C, t on the parents of the finer level's stored cells
      const long long tw = std::min<long long>(G.m, (a.gf.m + 1) / 2 + 1);
      bytes += sizeof(T) * (c_cells(G) + (double)nseg(l) * tw * tw * tw);
    }
    if (a.rmode >= 0)
      bytes += sizeof(T) * 2.0 * (a.rmode == 0 ? c_cells(G) / 8.0 : cube(H.geo[l - 1].n));
    run_shm(PRO == PRO_CORRECT ? "k_smooth_box<correct>" : "k_smooth_box<load>", bytes,
            dim3(nseg(l)), dim3(kBoxThreads), shm, k_smooth_box<T, PRO>, a);
  }

  void smooth_box(int l, const T* rhs, Geo gr, int nu, int pro, const T* d, const T* dt,
                  Geo gc, int fas, int rmode) {
    if (pro == PRO_CORRECT) smooth_box_pro<PRO_CORRECT>(l, rhs, gr, nu, d, dt, gc, 0, -1);
    else smooth_box_pro<PRO_LOAD>(l, rhs, gr, nu, d, dt, gc, fas, rmode);
  }

  // does the first smoothing pass of SR level l take the box path (and so
  // can form the FAS right-hand side and the restriction itself)?
  bool box_pass(int l, int nu) const { return nu > 0 && P->fused && box_fits(l); }

  // FMG interpolation onto the current copy of level l (streaming kernel)
  void interp(int l) {
    const Geo& G = H.geo[l];
    const Geo& Gc = H.geo[l - 1];
    int ce = G.ghost ? G.m : G.n;
    int zc = ce < 32 ? ce : 32;
    int ntz = (ce + zc - 1) / zc;
    run("k_interp_z", sizeof(T) * 1.125 * st_cells(G),
        grid_for((long long)ce * ce * ntz, nseg(l)), dim3(kBlock), k_interp_z<T>, H.u[l], G,
        (const T*)H.u[l - 1], Gc, zc, ce);
  }

  // prologue (none, FMG interpolation from level l-1, or the coarse-grid
  // correction from level l-1) followed by nu red-black sweeps on level l
  // returns true when the pass also restricted (rmode >= 0 on the box path)
  bool smooth(int l, const T* rhs, Geo gr, int nu, int pro = PRO_LOAD, int fas = 0,
              int rmode = -1) {
    lvl = l;
    const Geo& G = H.geo[l];
    const Geo& Gc = H.geo[l > 0 ? l - 1 : 0];
    // the coarse-grid correction adds w - t of level l-1 (formed per cell)
    const T* d = l > 0 ? H.u[l - 1] : nullptr;
    const T* dt = l > 0 ? H.t[l - 1] : nullptr;
    int st = 2 * nu;
    const bool boxp = st > 0 && P->fused && box_fits(l);
    // the first z pass forms the FMG interpolation itself, unless it is also
    // the pass that restricts
    const bool zint = pro == PRO_INTERP && !boxp && P->fused && st > 0 &&
                      !(seg_inplace(l) && rmode >= 0 && st <= 2);
    if (pro == PRO_INTERP && !zint) {
      interp(l);
      pro = PRO_LOAD;
    }
    if (boxp) {
      smooth_box(l, rhs, gr, nu, pro, d, dt, Gc, fas, rmode);
      return rmode >= 0 && pro != PRO_CORRECT;
    }
    if (fas && (pro != PRO_LOAD || !pass_fas(l)))
      throw hip_error("internal: FAS prologue requested off the box and column smoothers");
    if (st == 0 || !P->fused) {
      if (pro == PRO_CORRECT)
        run("k_correct", sizeof(T) * 2.25 * st_cells(G), grid_for(cube(G.m), nseg(l)),
            dim3(kBlock), k_correct<T>, H.u[l], G, d, dt, Gc);
      smooth_simple(l, rhs, gr, nu);
      return false;
    }
    bool first = true, restricted = false;
    const bool inpl = seg_inplace(l);
    const int mx = inpl ? 4 : P->max_stages;
    while (st > 0) {
      int ns = st >= mx ? mx : st;
      int pr = first ? pro : PRO_LOAD;
      // the solve's last pass may deliver the genuine cells itself
      double* out = nullptr;
      int om = 0;
      if (fin_out && inpl && st == ns && l == P->L - 1) {
        out = fin_out;
        om = fin_acc ? 2 : 1;
        fin_done = true;
      }
      if (pr == PRO_LOAD && rmode >= 0 && inpl && ns == 2 && st == ns && !om) {
        // the last pass of a pre-smoothing also restricts (residual epilogue)
        smooth_z<2, 2, PRO_LOAD, 1>(l, rhs, gr, d, dt, Gc, true, nullptr, 0, rmode);
        restricted = true;
      } else if (pr == PRO_LOAD && rmode == 0 && !inpl && nseg(l) == 1 && !cols_level(l) &&
                 ns == 2 && st == ns && sizeof(T) == 8 && P->zres) {
        // ... over two copies on a large global level (one more halo column)
        smooth_z<2, 2, PRO_LOAD, 1>(l, rhs, gr, d, dt, Gc, false, nullptr, 0, 0);
        restricted = true;
      } else if (pr == PRO_LOAD && rmode == 0 && !inpl && cols_level(l) && st == ns) {
        // ... and over two copies on the small global levels
        const int pf = first ? fas : 0;
        // four-stage passes with the epilogue load 2 (4 + 1) halo planes per
        // chunk: on 64^3 and up, 4-plane chunks (35 against 50 us at 64^3; at
        // 32^3, and for the other passes, 2-plane chunks are faster)
        if (ns == 2) smooth_cols<2, PRO_LOAD, 1>(l, rhs, gr, d, dt, Gc, pf);
        else if (G.n >= 64) smooth_cols<4, PRO_LOAD, 1, 4>(l, rhs, gr, d, dt, Gc, pf);
        else smooth_cols<4, PRO_LOAD, 1>(l, rhs, gr, d, dt, Gc, pf);
        restricted = true;
      } else if (pr == PRO_CORRECT) {
        smooth_z_ns<PRO_CORRECT>(ns, inpl, l, rhs, gr, d, dt, Gc, out, om);
      } else if (pr == PRO_INTERP) {
        smooth_z_ns<PRO_INTERP>(ns, inpl, l, rhs, gr, d, dt, Gc, out, om);
      } else {
        smooth_z_ns<PRO_LOAD>(ns, inpl, l, rhs, gr, d, dt, Gc, out, om, first ? fas : 0);
      }
      // a FAS prologue over two copies put the right-hand side in rf
      if (first && fas && !boxp) {
        rhs = H.rf[l];
        gr = G;
      }
      st -= ns;
      first = false;
    }
    return restricted;
  }

  // the persistent coarse-level kernel: FMG stages 0..top (mode 0) or one
  // V-cycle on level top with right-hand side rt (mode 1); fas: rt is the
  // restricted residual and the kernel forms the FAS right-hand side and t
  void coarse(int top, int mode, const T* rt, int fas = 0) {
    lvl = top;
    CoarseArgs<T> a;
    std::memset(&a, 0, sizeof a);
    double bytes = 0;
    for (int l = 0; l <= top; ++l) {
      a.u[l] = H.u[l];
      a.t[l] = H.t[l];
      a.r[l] = H.rhs[l];
      a.f[l] = H.f[l];
      a.n[l] = H.geo[l].n;
      bytes += 4.0 * sizeof(T) * cube(a.n[l]);
    }
    a.Ainv = P->Ainv;
    a.mm = P->n0 * P->n0 * P->n0;
    a.top = top;
    a.mode = mode;
    a.rt = rt;
    a.fas = mode == 1 ? fas : 0;
    if (a.fas) bytes += sizeof(T) * cube(a.n[top]);  // t written
    a.nu1 = P->nu1;
    a.nu2 = P->nu2;
    a.alpha = P->alpha;
    if (mode == 0 && checkpoints())
      for (int l = 0; l <= top; ++l) a.ck[l] = P->ck[l];
    size_t shm = coarse_layout(a.n, top, mode, a.mm, sizeof(T), a.ou, a.ot, a.orh, a.of, &a.ort,
                               &a.oai);
    if ((long long)shm + 1024 > P->lds_max) throw hip_error("internal: coarse levels exceed LDS");
    allow_lds((const void*)k_coarse<T>, P->lds_max - 1024);
    run_shm(mode == 0 ? "k_coarse<fmg>" : "k_coarse<vcycle>", bytes, dim3(1),
            dim3(kCoarseThreads), shm, k_coarse<T>, a);
  }



  // restriction of u and of the residual onto the coarse target cells
  // (skipped when the smoothing pass did it), then the coarse right-hand side
  // and t (skipped when the coarse level's first pass, or the coarse-level
  // kernel, forms them)
  void descend(int l, const T* rhs, Geo gr, int mode, int whole_f, bool restricted = false,
               bool rhs_deferred = false) {
    lvl = l;
    const Geo& G = H.geo[l];
    const Geo& Gc = H.geo[l - 1];
    int ns = nseg(l);
    int ce = mode == 0 ? cext(l) / 2 : Gc.n / P->S;
    double coarse = mode == 0 ? c_cells(G) / 8.0 : cube(Gc.n);
    double bytes = sizeof(T) * (16.0 * coarse + 2.0 * coarse);
    // a global level onto the whole coarse global level (rhs on the fine
    // level's own grid)
    const bool glob = !G.ghost && !Gc.ghost && !gr.ghost && gr.n == G.n && mode == 0 && G.n >= 4;
    if (restricted) {
      // done in the smoothing pass's epilogue
    } else if (P->fused && cube(ce) * ns > 300000) {
      // the streaming pass on large targets; small ones are latency bound and
      // take a one-thread-per-coarse-column march (global levels) or the
      // one-thread-per-coarse-cell kernel
      descend_z(l, rhs, gr, mode, ce, bytes);
    } else if (glob && P->fused) {
      const int nc = Gc.n, zc = 1;  // short chunks: latency bound
      run("k_resid_restrict_z", bytes,
          dim3((nc + kResTX - 1) / kResTX, (nc + kResTY - 1) / kResTY, (nc + zc - 1) / zc),
          dim3(kResTX * kResTY), k_resid_restrict_z<T>, (const T*)H.u[l], rhs, H.u[l - 1],
          H.rhs[l - 1], G.n, zc);
    } else {
      run("k_resid_restrict", bytes, grid_for(cube(ce), ns), dim3(kBlock), k_resid_restrict<T>,
          (const T*)H.u[l], G, rhs, gr, H.u[l - 1], H.rhs[l - 1], Gc, mode, ce);
    }
    if (rhs_deferred) return;
    int nsc = mode == 0 ? ns : 1;
    if (!Gc.ghost && whole_f && P->fused) {  // a global coarse level, F the whole level
      const int nc = Gc.n, zc = 2;  // short chunks: latency bound
      run("k_coarse_rhs_z", 4.0 * sizeof(T) * st_cells(Gc),
          dim3((nc + kResTX - 1) / kResTX, (nc + kResTY - 1) / kResTY, (nc + zc - 1) / zc),
          dim3(kResTX * kResTY), k_coarse_rhs_z<T>, (const T*)H.u[l - 1], H.rhs[l - 1],
          H.t[l - 1], nc, zc);
      return;
    }
    run("k_coarse_rhs", 4.0 * sizeof(T) * st_cells(Gc), grid_for(cube(Gc.m), nsc), dim3(kBlock),
        k_coarse_rhs<T>, (const T*)H.u[l - 1], H.rhs[l - 1], H.t[l - 1], Gc, G, whole_f);
  }

  // residual + restriction as one streaming pass (k_descend_z); ce is the
  // largest per-segment extent of the coarse target region
  void descend_z(int l, const T* rhs, Geo gr, int mode, int ce, double bytes) {
    constexpr int RY = 1, NC = kDescThreads * RY;
    const Geo& G = H.geo[l];
    DescArgs<T> a{};
    a.u = H.u[l];
    a.gu = G;
    a.rhs = rhs;
    a.gr = gr;
    a.uc = H.u[l - 1];
    a.rc = H.rhs[l - 1];
    a.gc = H.geo[l - 1];
    a.mode = mode;
    // tile shape: the fewest loaded fine columns covering the target
    long long best = -1;
    for (int tx = 1; tx <= ce && 2 * tx + 2 <= NC / 4; ++tx) {
      int ty = (NC / (2 * tx + 2) - 2) / 2;
      if (ty > ce) ty = ce;
      if (ty < 1) continue;
      long long cost = (long long)((ce + tx - 1) / tx) * ((ce + ty - 1) / ty) * (2 * tx + 2) *
                       (2 * ty + 2);
      if (tx < 8) cost += cost / 4;  // short rows load poorly
      if (best < 0 || cost <= best) {  // ties: the longer rows
        best = cost;
        a.ctx = tx;
        a.cty = ty;
      }
    }
    a.ntx = (ce + a.ctx - 1) / a.ctx;
    a.nty = (ce + a.cty - 1) / a.cty;
    int ns = nseg(l);
    long long bxy = (long long)a.ntx * a.nty * ns;
    int ntz = (int)(((P->target_blocks ? P->target_blocks : 1024) + bxy - 1) / bxy);
    // chunks of at least 8 coarse planes: each re-reads two halo fine planes
    int zmax = ce / 8 < 1 ? 1 : ce / 8;
    if (ntz > zmax) ntz = zmax;
    if (ntz < 1) ntz = 1;
    a.kc = (ce + ntz - 1) / ntz;
    a.ntz = (ce + a.kc - 1) / a.kc;
    a.nxcd = ns > 1 ? 1 : P->nxcd;
    int nt = a.ntx * a.nty * a.ntz;
    int per = (nt + a.nxcd - 1) / a.nxcd;
    run("k_descend_z", bytes, dim3(per * a.nxcd, ns), dim3(kDescThreads), k_descend_z<T, RY, 2>, a);
  }

  // FAS V-cycle on global level l with right-hand side rhs (Fig. 1)
  // presmoothed: S^nu1 has already been applied (fused with the FMG step),
  // and restricted tells whether that pass also restricted
  // fas: rhs holds the restricted residual only; the coarse kernel (levels up
  // to Lc) or the first pre-smoothing pass (column smoother) forms the FAS
  // right-hand side
  void vcycle_global(int l, const T* rhs, bool presmoothed = false, bool fas = false,
                     bool restricted = false) {
    if (l <= P->Lc) {
      coarse(l, 1, rhs, fas ? 1 : 0);
      return;
    }
    if (fas && (presmoothed || !pass_fas(l)))
      throw hip_error("internal: deferred FAS right-hand side without a pass to form it");
    const Geo& G = H.geo[l];
    if (!presmoothed) restricted = smooth(l, rhs, G, P->nu1, PRO_LOAD, fas ? 1 : 0, 0);
    if (fas) rhs = H.rf[l];  // the pre-smoothing formed the FAS right-hand side there
    const bool cf = l - 1 <= P->Lc || pass_fas(l - 1);
    descend(l, rhs, G, 0, 1, restricted, cf);
    vcycle_global(l - 1, H.rhs[l - 1], false, cf);
    smooth(l, rhs, G, P->nu2, PRO_CORRECT);
  }

  // SR V-cycle on segment level l inside the FMG stage whose top level is top
  // (Fig. 6); the top level's rhs is the global f_top read over C.
  // presmoothed: S^nu1 was applied by the caller (and restricted tells
  // whether that pass also restricted); fas: this level was just restricted
  // into and its first pass forms the FAS right-hand side and t.
  void vcycle_sr(int l, int top, bool presmoothed = false, bool restricted = false,
                 bool fas = false) {
    const Geo& G = H.geo[l];
    const T* rhs = (l == top) ? H.f[l] : H.rhs[l];
    Geo gr = (l == top) ? global_geo(G.n) : G;
    const int rmode = (l - 1 > P->T) ? 0 : 1;
    if (!presmoothed) restricted = smooth(l, rhs, gr, P->nu1, PRO_LOAD, fas ? 1 : 0, rmode);
    if (l - 1 > P->T) {
      const bool next_fas = box_pass(l - 1, P->nu1);
      descend(l, rhs, gr, 0, 0, restricted, next_fas);
      vcycle_sr(l - 1, top, false, false, next_fas);
    } else {
      const bool cf = l - 1 <= P->Lc || pass_fas(l - 1);
      descend(l, rhs, gr, 1, 1, restricted, cf);  // owner-computes transition restriction
      vcycle_global(l - 1, H.rhs[l - 1], false, cf);
    }
    if (l == P->L - 1) {  // the solve's last pass: deliver the genuine cells directly
      fin_out = want_out;
      fin_acc = want_acc;
    }
    smooth(l, rhs, gr, P->nu2, PRO_CORRECT);
    fin_out = nullptr;
  }

  // one FMG solve: ftop is the finest right-hand side (global N^3 of T);
  // the finest global u is H.u[L-1] (set by the caller when K == 0); with
  // K > 0 the genuine cells go to out (overwritten, or added when acc)
  void fmg(const T* ftop, double* out, int acc) {
    int L = P->L;
    H.f[L - 1] = const_cast<T*>(ftop);
    for (int l = 0; l < L; ++l) H.u[l] = H.ua[l];
    // f hierarchy down to the coarse-level kernel's top (it restricts
    // further): up to four levels per launch, reading each fine block once
    for (int l = L - 1; l > P->Lc;) {
      const int n = P->N >> (L - 1 - l);
      lvl = l;
      int d = l - P->Lc < 4 ? l - P->Lc : 4;
      while (d > 1 && n % (2 << d)) --d;
      if (d > 1) {
        double cells = 0;
        for (int k = 0; k <= d; ++k) cells += (double)cube(n >> k);
        run("k_restrict_chain", sizeof(T) * cells, dim3((unsigned)cube(n / (2 << d))), dim3(1024),
            k_restrict_chain<T>, (const T*)H.f[l], n, d, H.f[l - 1], H.f[l - 2],
            // (levels past depth are never written; any valid pointer)
            d > 2 ? H.f[l - 3] : H.f[l - 1], d > 3 ? H.f[l - 4] : H.f[l - 1]);
        l -= d;
      } else {
        run("k_restrict_global", sizeof(T) * 1.125 * cube(n), grid_for(cube(n / 2), 1),
            dim3(kBlock), k_restrict_global<T, T>, (const T*)H.f[l], n, H.f[l - 1]);
        --l;
      }
    }
    fin_done = false;
    want_out = P->K > 0 ? out : nullptr;
    want_acc = acc;
    // FMG stages on the coarse global levels in one launch
    coarse(P->Lc, 0, nullptr);
    for (int l = P->Lc + 1; l < L; ++l) {
      const Geo& G = H.geo[l];
      // Pi, S^alpha and the V-cycle's S^nu1 form one fused pass
      if (l <= P->T) {
        bool r = smooth(l, H.f[l], global_geo(G.n), P->alpha + P->nu1, PRO_INTERP, 0, 0);
        vcycle_global(l, H.f[l], true, false, r);
      } else {
        const int rmode = (l - 1 > P->T) ? 0 : 1;
        bool r = smooth(l, H.f[l], global_geo(G.n), P->alpha + P->nu1, PRO_INTERP, 0, rmode);
        vcycle_sr(l, l, true, r);
      }
      if (l < L - 1) checkpoint(l);
    }
    want_out = nullptr;
    if (P->K > 0 && !fin_done) {
      const Geo& G = H.geo[L - 1];
      lvl = L - 1;
      run("k_gather", (sizeof(T) + 8.0 + (acc ? 8.0 : 0.0)) * cube(P->N),
          grid_for(cube(G.g), nseg(L - 1)), dim3(kBlock), k_gather<T>, out, (const T*)H.u[L - 1],
          G, acc);
    }
  }
};

static void execute(fmg_plan* P, const double* f, double* u, hipStream_t s) {
  int N = P->N, L = P->L;
  long long cnt = cube(N);
  if (P->precision == FMG_FP64) {
    Exec<double> E{P, P->h64, s};
    E.dry = P->virt;
    if (P->K == 0) {
      // one copy of the finest level is the caller's u: start from the copy
      // that makes the last smoothing pass write into u
      double* ws = P->ws_finest;
      P->h64.ua[L - 1] = P->finest_odd ? ws : u;
      P->h64.ub[L - 1] = P->finest_odd ? u : ws;
    }
    if (!P->h64.ua[L - 1]) throw hip_error("internal: finest level has no storage");
    E.fmg(f, u, 0);
    if (!P->ck.empty() && P->ck[L - 1] && !P->virt)
      hipcheck(hipMemcpyAsync(P->ck[L - 1], u, sizeof(double) * (size_t)cnt,
                              hipMemcpyDeviceToDevice, s),
               "hipMemcpyAsync");
    return;
  }
  // mixed precision: u = FMG32(f); then refine times u += FMG32(f - L u)
  Exec<float> E{P, P->h32, s};
  E.dry = P->virt;
  for (int it = 0; it <= P->refine; ++it) {
    E.lvl = -1;
    const int zc = N >= 128 ? 16 : 8;
    E.run("k_resid64_to32", (it ? 20.0 : 12.0) * cnt,
          dim3((unsigned)((N + kResTX - 1) / kResTX), (unsigned)((N + kResTY - 1) / kResTY),
               (unsigned)((N + zc - 1) / zc)),
          dim3(kResTX * kResTY), k_resid64_to32, f, (const double*)u, (int)(it > 0), N, zc,
          P->r32);
    E.fmg(P->r32, u, it > 0);
    E.lvl = -1;
    if (P->K == 0)
      E.run("k_update64", (it ? 20.0 : 12.0) * cnt, grid_for(cnt, 1), dim3(kBlock),
            k_update64<float>, u, (const float*)P->h32.u[L - 1], cnt, (int)(it > 0));
  }
}

static void release(fmg_plan* P) {
  for (void* p : P->allocs) (void)hipFree(p);
  P->allocs.clear();
  delete P;
}

// Fill a plan: geometry, workspace (device memory, or virtual addresses for
// the schedule model) and the FP64 coarsest-level inverse.
// A dry walk of the schedule (after the geometry or the tuning changed):
// which copy of the finest global level holds the result last, so that the
// caller's u can be that copy?  (A one-level hierarchy is never smoothed.)
static void settle_schedule(fmg_plan* P) {
  if (P->precision != FMG_FP64 || P->K != 0) return;
  const int L = P->L;
  double* fake_u = (double*)(uintptr_t)(1ull << 41);
  double* keep_a = P->h64.ua[L - 1];
  double* keep_b = P->h64.ub[L - 1];
  const long long ml = P->model_launches;
  const double mb = P->model_bytes;
  const bool keep_virt = P->virt;
  P->virt = true;
  P->h64.ua[L - 1] = fake_u;  // stands for the caller's array
  P->h64.ub[L - 1] = P->ws_finest;
  {
    Exec<double> E{P, P->h64, nullptr};
    E.dry = true;
    E.fmg((const double*)(uintptr_t)(1ull << 40), fake_u, 0);
  }
  P->finest_odd = P->h64.u[L - 1] != fake_u;
  P->h64.ua[L - 1] = keep_a;
  P->h64.ub[L - 1] = keep_b;
  P->virt = keep_virt;
  P->model_launches = ml;
  P->model_bytes = mb;
}

static int32_t build_plan(int32_t N, const fmg_params* p, int device, bool virt, fmg_plan** out) {
  fmg_plan* P = new (std::nothrow) fmg_plan();
  if (!P) return fail(FMG_ENOMEM, "host allocation failed");
  P->virt = virt;
  P->lds_max = 160 * 1024;
  if (!virt) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device) == hipSuccess)
      P->lds_max = v;
    else
      (void)hipGetLastError();
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess &&
        v > 0)
      P->ncu = v;
    else
      (void)hipGetLastError();
  }
  P->N = N;
  P->L = p->levels;
  P->K = p->sr_levels;
  P->T = P->L - 1 - P->K;
  P->S = P->K > 0 ? p->segments_per_dim : 1;
  P->n0 = N >> (P->L - 1);
  P->device = device;
  P->nu1 = p->nu_pre;
  P->nu2 = p->nu_post;
  P->alpha = p->alpha;
  P->precision = p->precision;
  P->refine = p->refine_iters;
  P->J.assign(P->L, 0);
  for (int l = P->T + 1; l < P->L; ++l) P->J[l] = p->buffer_schedule[P->L - 1 - l];
  // coarse global levels: edge up to 16, at most the transition level, and
  // small enough for the LDS of one workgroup
  P->Lc = 0;
  {
    int nl[kCoarseMaxLevels];
    size_t esz = P->precision == FMG_FP64 ? sizeof(double) : sizeof(float);
    for (;;) {
      int c = P->Lc + 1;
      if (c > P->T || c >= kCoarseMaxLevels || (N >> (P->L - 1 - c)) > 16) break;
      for (int l = 0; l <= c; ++l) nl[l] = N >> (P->L - 1 - l);
      if (coarse_layout(nl, c, 0, P->n0 * P->n0 * P->n0, esz) + 1024 > (size_t)P->lds_max) break;
      ++P->Lc;
    }
  }
  std::vector<double> inv;
  if (!coarse_inverse(P->n0, inv)) {
    delete P;
    return fail(FMG_EINVAL, "singular coarsest matrix");
  }
  try {
    P->Ainv = (double*)dalloc(P, sizeof(double) * inv.size());
    if (P->precision == FMG_FP64) {
      build_hier(P, P->h64, true);
      if (P->K == 0) {
        P->ws_finest = P->h64.ub[P->L - 1];
        P->vpart = (double*)dalloc(P, sizeof(double) * (size_t)(2 * kNormMaxBlocks + 4));
      }
      settle_schedule(P);
    } else {
      build_hier(P, P->h32, false);
      P->r32 = (float*)dalloc(P, sizeof(float) * cube(N));
    }
    if (!virt) {
      // cells outside the domain and past a clipped box are never read; the
      // workspace still starts from zeros so every byte has a defined value
      for (size_t i = 0; i < P->allocs.size(); ++i)
        hipcheck(hipMemset(P->allocs[i], 0, P->sizes[i]), "hipMemset");
      hipcheck(hipMemcpy(P->Ainv, inv.data(), sizeof(double) * inv.size(), hipMemcpyHostToDevice),
               "hipMemcpy");
    }
  } catch (const std::bad_alloc&) {
    release(P);
    return fail(FMG_ENOMEM, "device allocation failed");
  } catch (const hip_error& ex) {
    release(P);
    return fail(FMG_EHIP, ex.what());
  }
  *out = P;
  return FMG_OK;
}

// ---------------------------------------------------------------------------
// C interface

// ---------------------------------------------------------------------------
// Batches: many independent solves (sizes may differ) spread over internal
// streams -- longest problems first, each to the least loaded stream -- so
// that small solves, each far from filling the GPU, run side by side.  The
// caller's stream forks to the internal streams and joins back, so the whole
// batch can be captured into one HIP graph and replayed with one launch.
// Problems on one stream run one after another and share a plan when their
// parameters and tuning agree.
struct fmg_batch {
  int device = 0;
  int count = 0;
  std::vector<int> N, plan_of, stream_of;
  std::vector<fmg_plan*> plans;
  std::vector<hipStream_t> streams;
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> join;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  long long bytes = 0;
};

static void batch_release(fmg_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  for (auto e : b->join) (void)hipEventDestroy(e);
  if (b->fork) (void)hipEventDestroy(b->fork);
  for (auto st : b->streams) (void)hipStreamDestroy(st);
  for (auto P : b->plans) release(P);
  delete b;
}

static bool same_params(const fmg_params& a, const fmg_params& b) {
  if (a.levels != b.levels || a.sr_levels != b.sr_levels ||
      a.segments_per_dim != b.segments_per_dim || a.nu_pre != b.nu_pre ||
      a.nu_post != b.nu_post || a.alpha != b.alpha || a.precision != b.precision ||
      a.refine_iters != b.refine_iters)
    return false;
  for (int i = 0; i < a.sr_levels; ++i)
    if (a.buffer_schedule[i] != b.buffer_schedule[i]) return false;
  return true;
}

static bool same_tuning(const fmg_tuning* a, const fmg_tuning* b) {
  if (!a || !b) return a == b;
  return a->max_stages == b->max_stages && a->seg_inplace == b->seg_inplace && a->box == b->box &&
         a->target_blocks == b->target_blocks && a->tile_x == b->tile_x;
}

// fork the caller's stream to the internal streams, enqueue every solve, join
static void batch_enqueue(fmg_batch* b, const double* const* f, double* const* u, hipStream_t s) {
  hipcheck(hipEventRecord(b->fork, s), "hipEventRecord");
  for (auto st : b->streams) hipcheck(hipStreamWaitEvent(st, b->fork, 0), "hipStreamWaitEvent");
  for (int i = 0; i < b->count; ++i) execute(b->plans[b->plan_of[i]], f[i], u[i], b->streams[b->stream_of[i]]);
  for (size_t k = 0; k < b->streams.size(); ++k) {
    hipcheck(hipEventRecord(b->join[k], b->streams[k]), "hipEventRecord");
    hipcheck(hipStreamWaitEvent(s, b->join[k], 0), "hipStreamWaitEvent");
  }
}

static std::string batch_check_io(const fmg_batch* b, const double* const* f, double* const* u) {
  if (!f || !u) return "f or u is NULL";
  for (int i = 0; i < b->count; ++i) {
    if (!f[i] || !u[i]) return "a problem's f or u is NULL";
    size_t bytes = sizeof(double) * (size_t)cube(b->N[i]);
    const char* fa = (const char*)f[i];
    const char* ua = (const char*)u[i];
    if (fa < ua + bytes && ua < fa + bytes) return "a problem's f and u overlap";
  }
  return "";
}

extern "C" {

const char* fmg_last_error(void) { return g_err.c_str(); }

int32_t fmg_check_params(int32_t N, const fmg_params* p) {
  std::string e = check(N, p);
  if (!e.empty()) return fail(FMG_EINVAL, e);
  return FMG_OK;
}

int32_t fmg_plan_create(int32_t N, const fmg_params* p, int32_t device, fmg_plan** out) {
  if (!out) return fail(FMG_EINVAL, "out is NULL");
  *out = nullptr;
  std::string e = check(N, p);
  if (!e.empty()) return fail(FMG_EINVAL, e);
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
    (void)hipGetLastError();
    return fail(FMG_EINVAL, "invalid device");
  }
  if (hipSetDevice(device) != hipSuccess) return fail(FMG_EHIP, "hipSetDevice failed");
  fmg_plan* P = nullptr;
  int32_t st = build_plan(N, p, device, false, &P);
  if (st == FMG_OK) *out = P;
  return st;
}

int32_t fmg_schedule_model(int32_t N, const fmg_params* p, fmg_schedule_stat* out) {
  if (!out) return fail(FMG_EINVAL, "out is NULL");
  std::string e = check(N, p);
  if (!e.empty()) return fail(FMG_EINVAL, e);
  fmg_plan* P = nullptr;
  int32_t st = build_plan(N, p, 0, true, &P);
  if (st != FMG_OK) return st;
  try {
    // two fake, distinct caller arrays
    const double* f = (const double*)(uintptr_t)(1ull << 40);
    double* u = (double*)(uintptr_t)(1ull << 41);
    P->model_launches = 0;
    P->model_bytes = 0;
    execute(P, f, u, nullptr);
    out->launches = P->model_launches;
    out->bytes = P->model_bytes;
    out->workspace_bytes = P->bytes;
  } catch (const hip_error& ex) {
    delete P;
    return fail(FMG_EHIP, ex.what());
  }
  delete P;
  return FMG_OK;
}

int32_t fmg_plan_execute(fmg_plan* P, const double* f, double* u, void* stream) {
  if (!P) return fail(FMG_EINVAL, "plan is NULL");
  if (!f || !u) return fail(FMG_EINVAL, "f or u is NULL");
  size_t bytes = sizeof(double) * (size_t)cube(P->N);
  const char* fa = (const char*)f;
  const char* ua = (const char*)u;
  if (fa < ua + bytes && ua < fa + bytes) return fail(FMG_EINVAL, "f and u overlap");
  try {
    hipcheck(hipSetDevice(P->device), "hipSetDevice");
    execute(P, f, u, (hipStream_t)stream);
  } catch (const hip_error& ex) {
    return fail(FMG_EHIP, ex.what());
  }
  return FMG_OK;
}

static int vcycle_solve(fmg_plan* P, const double* f, double* u, double rtol, int maxit,
                        double* relres, hipStream_t s);

int32_t fmg_plan_get_tuning(const fmg_plan* P, fmg_tuning* out) {
  if (!P || !out) return fail(FMG_EINVAL, "plan or out is NULL");
  out->max_stages = P->max_stages;
  out->seg_inplace = P->seg_inplace ? 1 : 0;
  out->box = P->use_box ? 1 : 0;
  out->target_blocks = (int32_t)P->target_blocks;
  out->tile_x = P->tile_x;
  return FMG_OK;
}

int32_t fmg_plan_set_tuning(fmg_plan* P, const fmg_tuning* t) {
  if (!P || !t) return fail(FMG_EINVAL, "plan or tuning is NULL");
  if (t->max_stages != 2 && t->max_stages != 4) return fail(FMG_EINVAL, "max_stages must be 2 or 4");
  if ((t->seg_inplace != 0 && t->seg_inplace != 1) || (t->box != 0 && t->box != 1))
    return fail(FMG_EINVAL, "seg_inplace and box must be 0 or 1");
  if (t->target_blocks != 0 && (t->target_blocks < 64 || t->target_blocks > 65536))
    return fail(FMG_EINVAL, "target_blocks must be 0 or in 64..65536");
  if (t->tile_x != 0 && (t->tile_x < 8 || t->tile_x > 256 || (t->tile_x & 1)))
    return fail(FMG_EINVAL, "tile_x must be 0 or even in 8..256");
  P->max_stages = t->max_stages;
  P->seg_inplace = t->seg_inplace != 0;
  P->use_box = t->box != 0;
  P->target_blocks = t->target_blocks;
  P->tile_x = t->tile_x;
  try {
    settle_schedule(P);
  } catch (const hip_error& ex) {
    return fail(FMG_EHIP, ex.what());
  }
  return FMG_OK;
}

int32_t fmg_plan_checkpoints(fmg_plan* P, double* const* out) {
  if (!P) return fail(FMG_EINVAL, "plan is NULL");
  if (P->precision != FMG_FP64) return fail(FMG_ENOTSUP, "checkpoints need an FP64 plan");
  if (!out) {
    P->ck.clear();
    return FMG_OK;
  }
  P->ck.assign(out, out + P->L);
  return FMG_OK;
}

int32_t fmg_plan_vcycles(fmg_plan* P, const double* f, double* u, double rtol, int32_t maxit,
                         int32_t* iters, double* relres, void* stream) {
  if (!P) return fail(FMG_EINVAL, "plan is NULL");
  if (!f || !u) return fail(FMG_EINVAL, "f or u is NULL");
  if (!(rtol >= 0.0) || maxit < 0) return fail(FMG_EINVAL, "rtol must be >= 0 and maxit >= 0");
  if (P->K != 0 || P->precision != FMG_FP64)
    return fail(FMG_ENOTSUP, "V-cycle iteration needs a global FP64 plan (sr_levels 0)");
  size_t bytes = sizeof(double) * (size_t)cube(P->N);
  const char* fa = (const char*)f;
  const char* ua = (const char*)u;
  if (fa < ua + bytes && ua < fa + bytes) return fail(FMG_EINVAL, "f and u overlap");
  try {
    hipcheck(hipSetDevice(P->device), "hipSetDevice");
    int it = vcycle_solve(P, f, u, rtol, maxit, relres, (hipStream_t)stream);
    if (it < 0) return fail(FMG_EINVAL, "the residual is not finite (NaN or Inf in f or u)");
    if (iters) *iters = it;
  } catch (const hip_error& ex) {
    return fail(FMG_EHIP, ex.what());
  }
  return FMG_OK;
}

int32_t fmg_plan_destroy(fmg_plan* P) {
  if (!P) return FMG_OK;
  (void)hipSetDevice(P->device);
  (void)hipDeviceSynchronize();
  release(P);
  return FMG_OK;
}

int32_t fmg_solve(const double* f, int32_t N, const fmg_params* p, double* u, void* stream) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(FMG_EHIP, "hipGetDevice failed");
  fmg_plan* P = nullptr;
  int32_t st = fmg_plan_create(N, p, dev, &P);
  if (st != FMG_OK) return st;
  st = fmg_plan_execute(P, f, u, stream);
  if (st == FMG_OK && hipStreamSynchronize((hipStream_t)stream) != hipSuccess)
    st = fail(FMG_EHIP, "hipStreamSynchronize failed");
  fmg_plan_destroy(P);
  return st;
}

int64_t fmg_plan_workspace_bytes(const fmg_plan* P) { return P ? P->bytes : 0; }

int32_t fmg_plan_profile(fmg_plan* P, int32_t enable) {
  if (!P) return fail(FMG_EINVAL, "plan is NULL");
  try {
    if (!P->prof.recs.empty()) {
      hipcheck(hipEventSynchronize(P->prof.recs.back().b), "hipEventSynchronize");
      P->prof.recycle();
    }
  } catch (const hip_error& ex) {
    return fail(FMG_EHIP, ex.what());
  }
  P->prof.on = enable != 0;
  return FMG_OK;
}

int32_t fmg_plan_profile_read(fmg_plan* P, fmg_kernel_stat* out, int32_t cap, int32_t* count) {
  if (!P || !count || (cap > 0 && !out)) return fail(FMG_EINVAL, "bad arguments");
  std::vector<fmg_kernel_stat> agg;
  try {
    if (!P->prof.recs.empty())
      hipcheck(hipEventSynchronize(P->prof.recs.back().b), "hipEventSynchronize");
    for (auto& r : P->prof.recs) {
      float ms = 0.f;
      hipcheck(hipEventElapsedTime(&ms, r.a, r.b), "hipEventElapsedTime");
      char key[64];
      if (r.level >= 0)
        std::snprintf(key, sizeof key, "%s@%d", r.name, r.level);
      else
        std::snprintf(key, sizeof key, "%s", r.name);
      size_t i = 0;
      while (i < agg.size() && std::strcmp(agg[i].name, key) != 0) ++i;
      if (i == agg.size()) {
        fmg_kernel_stat z;
        std::memset(&z, 0, sizeof z);
        std::snprintf(z.name, sizeof z.name, "%s", key);
        agg.push_back(z);
      }
      agg[i].launches += 1;
      agg[i].total_ms += ms;
      agg[i].bytes += r.bytes;
    }
    P->prof.recycle();
  } catch (const hip_error& ex) {
    return fail(FMG_EHIP, ex.what());
  }
  *count = (int32_t)agg.size();
  for (int32_t i = 0; i < cap && i < (int32_t)agg.size(); ++i) out[i] = agg[i];
  return FMG_OK;
}

// a10: norms of f - L u (mode 0), u - v (mode 1) or f (mode 2) into
// res[0..1] (device), with nb partial pairs in part (device)
static long long norm_blocks(int n) {
  long long nb = (cube(n) + kNormThreads - 1) / kNormThreads;
  return nb > kNormMaxBlocks ? kNormMaxBlocks : nb;
}

static hipError_t norms_launch(const double* a, const double* b, int n, int mode, double* part,
                               double* res, hipStream_t st) {
  const long long nb = norm_blocks(n);
  hipLaunchKernelGGL(k_norms, dim3((unsigned)nb), dim3(kNormThreads), 0, st, a, b, n, mode, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_norms_final, dim3(1), dim3(kNormThreads), 0, st, (const double*)part,
                     (int)nb, n, res);
  return hipGetLastError();
}

// the same, results copied to the host (synchronizes st)
static int32_t norms(const double* a, const double* b, int32_t n, int mode, double* out,
                     void* stream) {
  if (!a || !b || !out || n < 1) return fail(FMG_EINVAL, "bad arguments");
  if (a == b && mode == 0) return fail(FMG_EINVAL, "f and u must not be the same array");
  hipStream_t st = (hipStream_t)stream;
  const long long nb = norm_blocks(n);
  double* part = nullptr;
  if (hipMalloc(&part, sizeof(double) * (size_t)(2 * nb + 2)) != hipSuccess)
    return fail(FMG_ENOMEM, "hipMalloc failed");
  int32_t ret = FMG_OK;
  double res[2] = {0.0, 0.0};
  hipError_t e = norms_launch(a, b, n, mode, part, part + 2 * nb, st);
  if (e == hipSuccess) e = hipMemcpyAsync(res, part + 2 * nb, sizeof res, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) ret = fail(FMG_EHIP, hipGetErrorString(e));
  (void)hipFree(part);
  if (ret == FMG_OK) {
    out[0] = res[0];
    out[1] = res[1];
  }
  return ret;
}

// f4: V(nu1, nu2) cycles on the global hierarchy from the guess in u until
// max|f - L u| <= rtol max|f| or maxit cycles (the stopping rule of the
// oracle's iterated V-cycles); returns the cycle count, or -1 when the
// residual is not finite (NaN or Inf in f or u).  rtol == 0 runs exactly
// maxit cycles and forms the residual once, after the last, so that nothing
// waits on the host between cycles; with relres == NULL as well it forms no
// residual and never waits (every step is a launch or a device copy on s,
// so the call can be captured into a graph).  The norms' partials live in
// the plan.
static int vcycle_solve(fmg_plan* P, const double* f, double* u, double rtol, int maxit,
                        double* relres, hipStream_t s) {
  const int N = P->N, L = P->L;
  Hier<double>& H = P->h64;
  Exec<double> E{P, H, s};
  H.ua[L - 1] = u;
  H.ub[L - 1] = P->ws_finest;
  for (int l = 0; l < L; ++l) H.u[l] = H.ua[l];
  H.f[L - 1] = const_cast<double*>(f);
  if (!P->vpart) throw hip_error("internal: plan holds no norm partials");
  const long long nb = norm_blocks(N);
  double* part = P->vpart;
  double* res = part + 2 * nb;
  double h[4];
  const bool fixed = rtol == 0.0;
  if (fixed && !relres) {
    for (int it = 0; it < maxit; ++it) E.vcycle_global(L - 1, f);
    if (H.u[L - 1] != u)
      hipcheck(hipMemcpyAsync(u, H.u[L - 1], sizeof(double) * (size_t)cube(N),
                              hipMemcpyDeviceToDevice, s),
               "hipMemcpyAsync");
    return maxit;
  }
  hipcheck(norms_launch(f, f, N, 2, part, res + 2, s), "norms");
  int it = 0;
  double rn = 0.0, fn = 0.0;
  for (;;) {
    if (fixed && it < maxit) {
      E.vcycle_global(L - 1, f);
      ++it;
      continue;
    }
    hipcheck(norms_launch(f, H.u[L - 1], N, 0, part, res, s), "norms");
    hipcheck(hipMemcpyAsync(h, res, sizeof h, hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
    hipcheck(hipStreamSynchronize(s), "hipStreamSynchronize");
    rn = h[0];
    fn = h[2];
    if (!std::isfinite(rn) || !std::isfinite(fn)) return -1;
    if (fixed || rn <= rtol * fn || it >= maxit) break;
    E.vcycle_global(L - 1, f);
    ++it;
  }
  if (H.u[L - 1] != u)
    hipcheck(hipMemcpyAsync(u, H.u[L - 1], sizeof(double) * (size_t)cube(N),
                            hipMemcpyDeviceToDevice, s),
             "hipMemcpyAsync");
  hipcheck(hipStreamSynchronize(s), "hipStreamSynchronize");
  if (relres) *relres = fn > 0 ? rn / fn : rn;
  return it;
}

int32_t fmg_residual_norms(const double* f, const double* u, int32_t N, double* out,
                           void* stream) {
  return norms(f, u, N, 0, out, stream);
}

int32_t fmg_diff_norms(const double* u, const double* v, int32_t N, double* out, void* stream) {
  return norms(u, v, N, 1, out, stream);
}

// The allocation-free residual norms: the partial pairs live in `scratch`, a
// file-scope device array (one copy per GPU, held until the process ends).
// Host code never passes the array's name to a kernel: it is a host-side
// stand-in.  The device address comes from hipGetSymbolAddress, taken once per
// device with that device current, and is kept in scratch_dev.
constexpr int kScratchPairs = kNormMaxBlocks;
constexpr int kScratchMaxN = 4096;  // 4096^3 doubles already exceed one GPU's HBM
static __device__ __align__(256) double scratch[2 * kScratchPairs];
static std::mutex g_scratch_mu;
static std::vector<double*> g_scratch_dev;  // index: device ordinal

static hipError_t scratch_dev(int dev, double** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if ((int)g_scratch_dev.size() <= dev) g_scratch_dev.resize((size_t)dev + 1, nullptr);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_dev[dev] = (double*)p;
  }
  *out = g_scratch_dev[dev];
  return hipSuccess;
}

int32_t fmg_residual_norms_noalloc(const double* f, const double* u, int32_t N, double* out,
                                   void* stream) {
  if (!f || !u || !out || N < 1) return fail(FMG_EINVAL, "bad arguments");
  if (N > kScratchMaxN) return fail(FMG_EINVAL, "N exceeds 4096, the limit of the static scratch");
  if (f == u) return fail(FMG_EINVAL, "f and u must not be the same array");
  const long long nb = norm_blocks(N);
  if (nb > kScratchPairs)
    return fail(FMG_EINVAL, "the reduction needs more partials than the static scratch holds");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(FMG_EHIP, "hipGetDevice failed");
  double* part = nullptr;
  hipError_t e = scratch_dev(dev, &part);
  if (e != hipSuccess) return fail(FMG_EHIP, hipGetErrorString(e));
  // every partial pair the final reduction reads is written by this call's
  // first kernel, so nothing needs clearing
  e = norms_launch(f, u, N, 0, part, out, (hipStream_t)stream);
  return e == hipSuccess ? FMG_OK : fail(FMG_EHIP, hipGetErrorString(e));
}

int32_t fmg_op_apply(const double* u, int32_t n, double* out, void* stream) {
  if (!u || !out || n < 1) return fail(FMG_EINVAL, "bad arguments");
  Geo G = global_geo(n);
  hipLaunchKernelGGL((k_apply<double>), grid_for(cube(n), 1), dim3(kBlock), 0,
                     (hipStream_t)stream, u, G, out);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? FMG_OK : fail(FMG_EHIP, hipGetErrorString(e));
}

int32_t fmg_op_smooth(double* u, const double* rhs, int32_t n, int32_t nu, void* stream) {
  if (!u || !rhs || n < 1 || nu < 0) return fail(FMG_EINVAL, "bad arguments");
  // a one-level plan over the caller's arrays: the smoother runs exactly as
  // inside a solve; its second copy of u is a temporary buffer
  hipStream_t st = (hipStream_t)stream;
  double* tmp = nullptr;
  size_t bytes = sizeof(double) * (size_t)cube(n);
  if (hipMalloc(&tmp, bytes) != hipSuccess) return fail(FMG_ENOMEM, "hipMalloc failed");
  int32_t ret = FMG_OK;
  {
    fmg_plan P;
    P.N = n;
    P.L = 1;
    P.T = 0;
    P.h64.geo.assign(1, global_geo(n));
    P.h64.ua.assign(1, u);
    P.h64.ub.assign(1, tmp);
    P.h64.u.assign(1, u);
    P.h64.t.assign(1, nullptr);
    try {
      Exec<double> E{&P, P.h64, st};
      E.smooth(0, rhs, global_geo(n), nu);
      if (P.h64.u[0] != u)
        hipcheck(hipMemcpyAsync(u, tmp, bytes, hipMemcpyDeviceToDevice, st), "hipMemcpyAsync");
      hipcheck(hipStreamSynchronize(st), "hipStreamSynchronize");
    } catch (const hip_error& ex) {
      ret = fail(FMG_EHIP, ex.what());
    }
  }
  (void)hipFree(tmp);
  return ret;
}

int32_t fmg_op_restrict(const double* fine, int32_t n, double* coarse, void* stream) {
  if (!fine || !coarse || n < 2 || (n & 1)) return fail(FMG_EINVAL, "bad arguments");
  hipLaunchKernelGGL((k_restrict_global<double, double>), grid_for(cube(n / 2), 1), dim3(kBlock),
                     0, (hipStream_t)stream, fine, n, coarse);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? FMG_OK : fail(FMG_EHIP, hipGetErrorString(e));
}

int32_t fmg_op_interp(const double* coarse, int32_t n, double* fine, void* stream) {
  if (!fine || !coarse || n < 1) return fail(FMG_EINVAL, "bad arguments");
  Geo Gf = global_geo(2 * n), Gc = global_geo(n);
  int ce = 2 * n, zc = ce < 32 ? ce : 32, ntz = (ce + zc - 1) / zc;
  hipLaunchKernelGGL((k_interp_z<double>), grid_for((long long)ce * ce * ntz, 1), dim3(kBlock), 0,
                     (hipStream_t)stream, fine, Gf, coarse, Gc, zc, ce);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? FMG_OK : fail(FMG_EHIP, hipGetErrorString(e));
}

int32_t fmg_batch_create(int32_t count, const int32_t* N, const fmg_params* params,
                         const fmg_tuning* tuning, int32_t nstreams, int32_t device,
                         fmg_batch** out) {
  if (!out) return fail(FMG_EINVAL, "out is NULL");
  *out = nullptr;
  if (count < 1 || !N || !params) return fail(FMG_EINVAL, "count, N or params invalid");
  if (nstreams < 1 || nstreams > 16) return fail(FMG_EINVAL, "streams must be in 1..16");
  for (int i = 0; i < count; ++i) {
    std::string e = check(N[i], &params[i]);
    if (!e.empty()) return fail(FMG_EINVAL, "problem " + std::to_string(i) + ": " + e);
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
    (void)hipGetLastError();
    return fail(FMG_EINVAL, "invalid device");
  }
  if (hipSetDevice(device) != hipSuccess) return fail(FMG_EHIP, "hipSetDevice failed");
  fmg_batch* b = new (std::nothrow) fmg_batch();
  if (!b) return fail(FMG_ENOMEM, "host allocation failed");
  b->device = device;
  b->count = count;
  b->N.assign(N, N + count);
  b->plan_of.assign(count, -1);
  b->stream_of.assign(count, 0);
  const int ns = nstreams < count ? nstreams : count;
  // longest problems first, each to the least loaded stream
  std::vector<int> order(count);
  for (int i = 0; i < count; ++i) order[i] = i;
  std::sort(order.begin(), order.end(), [&](int a, int c) {
    return cube(N[a]) != cube(N[c]) ? cube(N[a]) > cube(N[c]) : a < c;
  });
  std::vector<double> load(ns, 0.0);
  for (int i : order) {
    int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    b->stream_of[i] = k;
    load[k] += (double)cube(N[i]) * (params[i].precision == FMG_FP64 ? 1.0 : 2.0);
  }
  try {
    for (int k = 0; k < ns; ++k) {
      hipStream_t st;
      hipcheck(hipStreamCreateWithFlags(&st, hipStreamNonBlocking), "hipStreamCreate");
      b->streams.push_back(st);
      hipEvent_t e;
      hipcheck(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate");
      b->join.push_back(e);
    }
    hipcheck(hipEventCreateWithFlags(&b->fork, hipEventDisableTiming), "hipEventCreate");
    // one plan per (stream, N, parameters, tuning)
    std::vector<int> owner;  // problem that defined each plan
    for (int i = 0; i < count; ++i) {
      const fmg_tuning* ti = tuning ? &tuning[i] : nullptr;
      for (size_t j = 0; j < owner.size(); ++j) {
        const int o = owner[j];
        if (b->stream_of[o] == b->stream_of[i] && N[o] == N[i] && same_params(params[o], params[i]) &&
            same_tuning(tuning ? &tuning[o] : nullptr, ti)) {
          b->plan_of[i] = (int)j;
          break;
        }
      }
      if (b->plan_of[i] >= 0) continue;
      fmg_plan* P = nullptr;
      int32_t st = build_plan(N[i], &params[i], device, false, &P);
      if (st != FMG_OK) {
        std::string msg = "problem " + std::to_string(i) + ": " + g_err;
        batch_release(b);
        return fail(st, msg);
      }
      b->plans.push_back(P);
      b->bytes += P->bytes;
      if (ti) {
        st = fmg_plan_set_tuning(P, ti);
        if (st != FMG_OK) {
          std::string msg = "problem " + std::to_string(i) + ": " + g_err;
          batch_release(b);
          return fail(st, msg);
        }
      }
      b->plan_of[i] = (int)b->plans.size() - 1;
      owner.push_back(i);
    }
  } catch (const hip_error& ex) {
    batch_release(b);
    return fail(FMG_EHIP, ex.what());
  }
  *out = b;
  return FMG_OK;
}

int32_t fmg_batch_execute(fmg_batch* b, const double* const* f, double* const* u, void* stream) {
  if (!b) return fail(FMG_EINVAL, "batch is NULL");
  std::string e = batch_check_io(b, f, u);
  if (!e.empty()) return fail(FMG_EINVAL, e);
  try {
    hipcheck(hipSetDevice(b->device), "hipSetDevice");
    batch_enqueue(b, f, u, (hipStream_t)stream);
  } catch (const hip_error& ex) {
    return fail(FMG_EHIP, ex.what());
  }
  return FMG_OK;
}

int32_t fmg_batch_capture(fmg_batch* b, const double* const* f, double* const* u, void* stream) {
  if (!b) return fail(FMG_EINVAL, "batch is NULL");
  if (!stream) return fail(FMG_EINVAL, "capture needs a non-default stream");
  std::string e = batch_check_io(b, f, u);
  if (!e.empty()) return fail(FMG_EINVAL, e);
  hipStream_t s = (hipStream_t)stream;
  for (auto P : b->plans)
    if (P->prof.on) return fail(FMG_EINVAL, "disable plan profiling before capture");
  try {
    hipcheck(hipSetDevice(b->device), "hipSetDevice");
    if (b->exec) hipcheck(hipGraphExecDestroy(b->exec), "hipGraphExecDestroy");
    if (b->graph) hipcheck(hipGraphDestroy(b->graph), "hipGraphDestroy");
    b->exec = nullptr;
    b->graph = nullptr;
    hipcheck(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    try {
      batch_enqueue(b, f, u, s);
    } catch (...) {
      hipGraph_t g = nullptr;
      (void)hipStreamEndCapture(s, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    hipcheck(hipStreamEndCapture(s, &b->graph), "hipStreamEndCapture");
    hipcheck(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0), "hipGraphInstantiate");
  } catch (const hip_error& ex) {
    return fail(FMG_EHIP, ex.what());
  }
  return FMG_OK;
}

int32_t fmg_batch_replay(fmg_batch* b, void* stream) {
  if (!b) return fail(FMG_EINVAL, "batch is NULL");
  if (!b->exec) return fail(FMG_EINVAL, "nothing captured");
  hipError_t e = hipSetDevice(b->device);
  if (e == hipSuccess) e = hipGraphLaunch(b->exec, (hipStream_t)stream);
  return e == hipSuccess ? FMG_OK : fail(FMG_EHIP, hipGetErrorString(e));
}

int64_t fmg_batch_workspace_bytes(const fmg_batch* b) { return b ? b->bytes : 0; }

int32_t fmg_batch_destroy(fmg_batch* b) {
  if (!b) return FMG_OK;
  (void)hipSetDevice(b->device);
  (void)hipDeviceSynchronize();
  batch_release(b);
  return FMG_OK;
}

}  // extern "C"
