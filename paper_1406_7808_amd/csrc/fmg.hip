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

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/fmg.h"
#include "grid.hpp"
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

#define LAUNCH_CHECK(name) hipcheck(hipGetLastError(), name)

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
};

struct fmg_plan {
  int N = 0, L = 0, K = 0, T = 0, S = 1, n0 = 1, device = 0;
  int nu1 = 2, nu2 = 2, alpha = 1, precision = FMG_FP64, refine = 2;
  std::vector<int> J;  // J[l] for SR levels, indexed by level
  Hier<double> h64;
  Hier<float> h32;
  double* Ainv = nullptr;
  float* r32 = nullptr;  // FP32 right-hand side of the inner solves
  std::vector<void*> allocs;
  std::vector<size_t> sizes;
  long long bytes = 0;
};

static void* dalloc(fmg_plan* P, size_t bytes) {
  void* p = nullptr;
  if (bytes == 0) return nullptr;
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

template <class T>
static void build_hier(fmg_plan* P, Hier<T>& H, bool finest_external) {
  int L = P->L;
  H.geo.resize(L);
  H.u.assign(L, nullptr);
  H.t.assign(L, nullptr);
  H.rhs.assign(L, nullptr);
  H.f.assign(L, nullptr);
  for (int l = 0; l < L; ++l) {
    int n = P->N >> (L - 1 - l);
    bool sr = l > P->T;
    H.geo[l] = sr ? segment_geo(n, P->S, P->J[l]) : global_geo(n);
    long long cnt = sr ? cube(P->S) * H.geo[l].sstride : cube(n);
    if (l < L - 1) H.f[l] = (T*)dalloc(P, sizeof(T) * cube(n));
    if (l == L - 1 && !sr && finest_external) continue;  // caller's array
    H.u[l] = (T*)dalloc(P, sizeof(T) * cnt);
    if (l < L - 1) {
      H.t[l] = (T*)dalloc(P, sizeof(T) * cnt);
      H.rhs[l] = (T*)dalloc(P, sizeof(T) * cnt);
    }
  }
}

// ---------------------------------------------------------------------------
// schedule

static const int kBlock = 256;

static dim3 grid_for(long long cells, int nseg) {
  return dim3((unsigned)((cells + kBlock - 1) / kBlock), (unsigned)nseg);
}

template <class T>
struct Exec {
  using A = T;  // smoothing arithmetic: FP64 or FP32
  fmg_plan* P;
  Hier<T>& H;
  hipStream_t s;

  int nseg(int l) const { return l > P->T ? P->S * P->S * P->S : 1; }
  int cext(int l) const {  // maximal compute-region edge
    const Geo& G = H.geo[l];
    return (G.g + 2 * G.J) < G.n ? (G.g + 2 * G.J) : G.n;
  }

  void smooth(int l, const T* rhs, Geo gr, int nu) {
    const Geo& G = H.geo[l];
    double h = 1.0 / (double)G.n;
    A h2 = (A)(h * h);
    int ce = cext(l);
    for (int it = 0; it < nu; ++it)
      for (int col = 0; col < 2; ++col) {
        hipLaunchKernelGGL((k_gs_half<T, A>), grid_for(cube(ce), nseg(l)), dim3(kBlock), 0, s,
                           H.u[l], G, rhs, gr, col, h2, ce);
        LAUNCH_CHECK("k_gs_half");
      }
  }

  void coarse_solve(T* u0, const T* rhs0) {
    hipLaunchKernelGGL((k_coarse_solve<T>), dim3(1), dim3(kBlock), 0, s, u0, rhs0, P->Ainv,
                       P->n0 * P->n0 * P->n0);
    LAUNCH_CHECK("k_coarse_solve");
  }

  // FAS V-cycle on global level l with right-hand side rhs (Fig. 1)
  void vcycle_global(int l, const T* rhs) {
    if (l == 0) {
      coarse_solve(H.u[0], rhs);
      return;
    }
    const Geo& G = H.geo[l];
    const Geo& Gc = H.geo[l - 1];
    smooth(l, rhs, G, P->nu1);
    hipLaunchKernelGGL((k_resid_restrict<T>), grid_for(cube(G.n / 2), 1), dim3(kBlock), 0, s,
                       H.u[l], G, rhs, G, H.u[l - 1], H.rhs[l - 1], Gc, 0, G.n / 2);
    LAUNCH_CHECK("k_resid_restrict");
    hipLaunchKernelGGL((k_coarse_rhs<T>), grid_for(cube(Gc.m), 1), dim3(kBlock), 0, s,
                       H.u[l - 1], H.rhs[l - 1], H.t[l - 1], Gc, G, 1);
    LAUNCH_CHECK("k_coarse_rhs");
    vcycle_global(l - 1, H.rhs[l - 1]);
    hipLaunchKernelGGL((k_correct<T>), grid_for(cube(G.m), 1), dim3(kBlock), 0, s, H.u[l], G,
                       H.u[l - 1], H.t[l - 1], Gc);
    LAUNCH_CHECK("k_correct");
    smooth(l, rhs, G, P->nu2);
  }

  // SR V-cycle on segment level l inside the FMG stage whose top level is top
  // (Fig. 6); the top level's rhs is the global f_top read over C
  void vcycle_sr(int l, int top) {
    const Geo& G = H.geo[l];
    const Geo& Gc = H.geo[l - 1];
    const T* rhs = (l == top) ? H.f[l] : H.rhs[l];
    Geo gr = (l == top) ? global_geo(G.n) : G;
    int ns = nseg(l);
    smooth(l, rhs, gr, P->nu1);
    if (l - 1 > P->T) {
      int ce = cext(l) / 2;
      hipLaunchKernelGGL((k_resid_restrict<T>), grid_for(cube(ce), ns), dim3(kBlock), 0, s,
                         H.u[l], G, rhs, gr, H.u[l - 1], H.rhs[l - 1], Gc, 0, ce);
      LAUNCH_CHECK("k_resid_restrict");
      hipLaunchKernelGGL((k_coarse_rhs<T>), grid_for(cube(Gc.m), ns), dim3(kBlock), 0, s,
                         H.u[l - 1], H.rhs[l - 1], H.t[l - 1], Gc, G, 0);
      LAUNCH_CHECK("k_coarse_rhs");
      vcycle_sr(l - 1, top);
    } else {
      int e = Gc.n / P->S;
      hipLaunchKernelGGL((k_resid_restrict<T>), grid_for(cube(e), ns), dim3(kBlock), 0, s,
                         H.u[l], G, rhs, gr, H.u[l - 1], H.rhs[l - 1], Gc, 1, e);
      LAUNCH_CHECK("k_resid_restrict");
      hipLaunchKernelGGL((k_coarse_rhs<T>), grid_for(cube(Gc.m), 1), dim3(kBlock), 0, s,
                         H.u[l - 1], H.rhs[l - 1], H.t[l - 1], Gc, G, 1);
      LAUNCH_CHECK("k_coarse_rhs");
      vcycle_global(l - 1, H.rhs[l - 1]);
    }
    hipLaunchKernelGGL((k_correct<T>), grid_for(cube(G.m), ns), dim3(kBlock), 0, s, H.u[l], G,
                       H.u[l - 1], H.t[l - 1], Gc);
    LAUNCH_CHECK("k_correct");
    smooth(l, rhs, gr, P->nu2);
  }

  // one FMG solve: ftop is the finest right-hand side (global N^3 of T);
  // the finest global u is H.u[L-1] (set by the caller when K == 0); with
  // K > 0 the genuine cells go to out (overwritten, or added when acc)
  void fmg(const T* ftop, double* out, int acc) {
    int L = P->L;
    H.f[L - 1] = const_cast<T*>(ftop);
    for (int l = L - 1; l > 0; --l) {
      int n = P->N >> (L - 1 - l);
      hipLaunchKernelGGL((k_restrict_global<T, T>), grid_for(cube(n / 2), 1), dim3(kBlock), 0, s,
                         H.f[l], n, H.f[l - 1]);
      LAUNCH_CHECK("k_restrict_global");
    }
    coarse_solve(H.u[0], H.f[0]);
    for (int l = 1; l < L; ++l) {
      const Geo& G = H.geo[l];
      const Geo& Gc = H.geo[l - 1];
      int ns = nseg(l);
      hipLaunchKernelGGL((k_interp<T>), grid_for(cube(G.m), ns), dim3(kBlock), 0, s, H.u[l], G,
                         H.u[l - 1], Gc);
      LAUNCH_CHECK("k_interp");
      smooth(l, H.f[l], global_geo(G.n), P->alpha);
      if (l <= P->T)
        vcycle_global(l, H.f[l]);
      else
        vcycle_sr(l, l);
    }
    if (P->K > 0) {
      const Geo& G = H.geo[L - 1];
      hipLaunchKernelGGL((k_gather<T>), grid_for(cube(G.g), nseg(L - 1)), dim3(kBlock), 0, s, out,
                         H.u[L - 1], G, acc);
      LAUNCH_CHECK("k_gather");
    }
  }
};

static void execute(fmg_plan* P, const double* f, double* u, hipStream_t s) {
  int N = P->N, L = P->L;
  long long cnt = cube(N);
  if (P->precision == FMG_FP64) {
    Exec<double> E{P, P->h64, s};
    if (P->K == 0) P->h64.u[L - 1] = u;
    E.fmg(f, u, 0);
    return;
  }
  // mixed precision: u = FMG32(f); then refine times u += FMG32(f - L u)
  Exec<float> E{P, P->h32, s};
  for (int it = 0; it <= P->refine; ++it) {
    hipLaunchKernelGGL(k_resid64_to32, grid_for(cnt, 1), dim3(kBlock), 0, s, f,
                       it == 0 ? (const double*)nullptr : (const double*)u, N, P->r32);
    LAUNCH_CHECK("k_resid64_to32");
    E.fmg(P->r32, u, it > 0);
    if (P->K == 0) {
      hipLaunchKernelGGL((k_update64<float>), grid_for(cnt, 1), dim3(kBlock), 0, s, u,
                         P->h32.u[L - 1], cnt, it > 0);
      LAUNCH_CHECK("k_update64");
    }
  }
}

static void release(fmg_plan* P) {
  for (void* p : P->allocs) (void)hipFree(p);
  P->allocs.clear();
  delete P;
}

// ---------------------------------------------------------------------------
// C interface

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
  fmg_plan* P = new (std::nothrow) fmg_plan();
  if (!P) return fail(FMG_ENOMEM, "host allocation failed");
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
  std::vector<double> inv;
  if (!coarse_inverse(P->n0, inv)) {
    delete P;
    return fail(FMG_EINVAL, "singular coarsest matrix");
  }
  try {
    if (P->precision == FMG_FP64) {
      build_hier(P, P->h64, true);
    } else {
      build_hier(P, P->h32, false);
      P->r32 = (float*)dalloc(P, sizeof(float) * cube(N));
    }
    P->Ainv = (double*)dalloc(P, sizeof(double) * inv.size());
    // cells outside the domain and past a clipped box are never read; the
    // workspace still starts from zeros so every byte has a defined value
    for (size_t i = 0; i < P->allocs.size(); ++i)
      hipcheck(hipMemset(P->allocs[i], 0, P->sizes[i]), "hipMemset");
    hipcheck(hipMemcpy(P->Ainv, inv.data(), sizeof(double) * inv.size(), hipMemcpyHostToDevice),
             "hipMemcpy");
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
  Geo G = global_geo(n);
  double h = 1.0 / (double)n;
  for (int it = 0; it < nu; ++it)
    for (int col = 0; col < 2; ++col)
      hipLaunchKernelGGL((k_gs_half<double, double>), grid_for(cube(n), 1), dim3(kBlock), 0,
                         (hipStream_t)stream, u, G, rhs, G, col, h * h, n);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? FMG_OK : fail(FMG_EHIP, hipGetErrorString(e));
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
  hipLaunchKernelGGL((k_interp<double>), grid_for(cube(2 * n), 1), dim3(kBlock), 0,
                     (hipStream_t)stream, fine, Gf, coarse, Gc);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? FMG_OK : fail(FMG_EHIP, hipGetErrorString(e));
}

}  // extern "C"
