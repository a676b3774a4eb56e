// Krylov solvers on the device: unpreconditioned BiCGSTAB (van der Vorst; the
// paper's solver follows Eigen's BiCGSTAB, Sec. 5.4) in FP64 or FP32, and
// mixed precision: FP32 BiCGSTAB with reliable updates (the partial solution
// is added into the FP64 one and the FP32 recurrence restarts from the FP64
// true residual), finished in FP64 where FP32 stops making progress.
//
// The recurrence scalars live in device memory.  Every reduction kernel
// writes one partial sum per workgroup; the last workgroup to finish (found
// with a device-scope fence and an atomic counter) adds the partials in a
// fixed order and updates the scalars, so results are bitwise reproducible
// and the host only reads the scalars every `check_every` iterations.  The
// check_every iterations can be captured once into a hipGraph and replayed.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <memory>
#include <type_traits>

#include "cpm_internal.hpp"

namespace cpm {

struct Scal {
  double rho, rho_old, alpha, omega, beta;
  double bb, rr, tol2;
  double d0, d1;
  int done, breakdown, it, restarts;
  unsigned counter;
  unsigned pad;
};

constexpr int kRedThreads = 256;
constexpr int kMaxParts = 1024;

static int red_grid(int64_t n) {
  int64_t g = (n + kRedThreads * 4 - 1) / (kRedThreads * 4);
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, kMaxParts));
}

// Workgroup sum of NR values; thread 0 gets the totals.
template <int NR>
__device__ __forceinline__ void wg_sum(double v[NR], double (*sh)[kRedThreads]) {
  for (int k = 0; k < NR; ++k) sh[k][threadIdx.x] = v[k];
  __syncthreads();
  for (int o = kRedThreads / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o)
      for (int k = 0; k < NR; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + o];
    __syncthreads();
  }
  for (int k = 0; k < NR; ++k) v[k] = sh[k][0];
}

// Writes this workgroup's partials; returns true in every thread of the last
// workgroup, with out[] holding the grand totals (fixed summation order).
template <int NR>
__device__ bool finish_reduction(double v[NR], double* part, Scal* S, double out[NR]) {
  __shared__ double sh[NR][kRedThreads];
  __shared__ bool last;
  wg_sum<NR>(v, sh);
  if (threadIdx.x == 0) {
    for (int k = 0; k < NR; ++k) part[k * kMaxParts + blockIdx.x] = v[k];
    __threadfence();
    const unsigned prev = atomicAdd(&S->counter, 1u);
    last = prev == gridDim.x - 1;
  }
  __syncthreads();
  if (!last) return false;
  __threadfence();
  double acc[NR];
  for (int k = 0; k < NR; ++k) acc[k] = 0.0;
  for (int i = threadIdx.x; i < (int)gridDim.x; i += kRedThreads)
    for (int k = 0; k < NR; ++k) acc[k] += __builtin_nontemporal_load(&part[k * kMaxParts + i]);
  __syncthreads();
  wg_sum<NR>(acc, sh);
  for (int k = 0; k < NR; ++k) out[k] = acc[k];
  if (threadIdx.x == 0) S->counter = 0;
  return true;
}

// r = b - v;  rh = r;  p = r;  sums (rh, r), (r, r), (b, b)
template <class T>
__global__ __launch_bounds__(256) void k_init(int64_t n, const T* __restrict__ b, const T* __restrict__ v,
                                              bool has_v, T* r, T* rh, T* p, double* part, Scal* S,
                                              double tol) {
  double acc[2] = {0.0, 0.0};
  for (int64_t i = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kRedThreads) {
    const T ri = has_v ? b[i] - v[i] : b[i];
    r[i] = ri;
    rh[i] = ri;
    p[i] = ri;
    const double d = (double)ri, bd = (double)b[i];
    acc[0] += d * d;
    acc[1] += bd * bd;
  }
  double tot[2];
  if (finish_reduction<2>(acc, part, S, tot) && threadIdx.x == 0) {
    S->rho = tot[0];
    S->rho_old = tot[0];
    S->rr = tot[0];
    S->bb = tot[1];
    S->tol2 = tol * tol * tot[1];
    S->alpha = S->omega = 1.0;
    S->beta = 0.0;
    S->breakdown = 0;
    S->done = (tot[0] <= S->tol2) ? 1 : 0;
  }
}

// Finishes a dot product fused into the apply that produced v (partials of
// (y, v) in dp[0 .. np) and of (v, v) in dp[np .. 2 np)).  MODE 0: y = rh,
// alpha = rho / (rh, v).  MODE 1: y = s, v = t, omega = (t, s) / (t, t).
template <int MODE>
__global__ __launch_bounds__(256) void k_dot_fin(const double* __restrict__ dp, int np,
                                                 double* part, Scal* S) {
  if (S->done) return;
  double acc[2] = {0.0, 0.0};
  for (int i = blockIdx.x * kRedThreads + threadIdx.x; i < np; i += gridDim.x * kRedThreads) {
    acc[0] += dp[i];
    acc[1] += dp[np + i];
  }
  double tot[2];
  if (finish_reduction<2>(acc, part, S, tot) && threadIdx.x == 0) {
    if (MODE == 0) {
      if (tot[0] == 0.0 || !__builtin_isfinite(tot[0])) {
        S->breakdown = 1;
        S->done = 1;
      } else {
        S->alpha = S->rho / tot[0];
      }
    } else {
      if (tot[1] == 0.0 || !__builtin_isfinite(tot[1])) {
        S->omega = 0.0;
      } else {
        S->omega = tot[0] / tot[1];
      }
    }
  }
}

// s = r - alpha v
template <class T>
__global__ __launch_bounds__(256) void k_s(int64_t n, const T* __restrict__ r, const T* __restrict__ v,
                                           T* __restrict__ s, const Scal* S) {
  if (S->done) return;
  const T al = (T)S->alpha;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    s[i] = r[i] - al * v[i];
}

// x += alpha p + omega s;  r = s - omega t;  rho = (rh, r);  rr = (r, r).
// The iterate x may be kept in a wider type TX than the recurrence vectors
// (FP64 x with an FP32 recurrence: the update is not rounded to FP32).
template <class T, class TX>
__global__ __launch_bounds__(256) void k_xr(int64_t n, TX* __restrict__ x, const T* __restrict__ p,
                                            const T* __restrict__ s, const T* __restrict__ t,
                                            T* __restrict__ r, const T* __restrict__ rh,
                                            double* part, Scal* S) {
  if (S->done) return;
  const T al = (T)S->alpha, om = (T)S->omega;
  const TX alx = (TX)S->alpha, omx = (TX)S->omega;
  double acc[2] = {0.0, 0.0};
  for (int64_t i = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kRedThreads) {
    const T si = s[i];
    x[i] = x[i] + alx * (TX)p[i] + omx * (TX)si;
    const T ri = si - om * t[i];
    r[i] = ri;
    acc[0] += (double)rh[i] * (double)ri;
    acc[1] += (double)ri * (double)ri;
  }
  double tot[2];
  if (finish_reduction<2>(acc, part, S, tot) && threadIdx.x == 0) {
    S->it += 1;
    S->rr = tot[1];
    if (!__builtin_isfinite(tot[1])) {
      S->breakdown = 1;
      S->done = 1;
    } else if (tot[0] == 0.0 || S->omega == 0.0) {
      S->done = 1;
      S->breakdown = tot[1] <= S->tol2 ? 0 : 1;
    } else {
      // rho and beta are kept current also on the converging iteration
      S->rho_old = S->rho;
      S->rho = tot[0];
      S->beta = (S->rho / S->rho_old) * (S->alpha / S->omega);
      if (tot[1] <= S->tol2) S->done = 1;
    }
  }
}

template <class T>
__global__ void k_zero(int64_t n, T* __restrict__ x) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] = T(0);
}

// p = r + beta (p - omega v)
template <class T>
__global__ __launch_bounds__(256) void k_p(int64_t n, const T* __restrict__ r, T* __restrict__ p,
                                           const T* __restrict__ v, const Scal* S) {
  if (S->done) return;
  const T be = (T)S->beta, om = (T)S->omega;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = r[i] + be * (p[i] - om * v[i]);
}

// ---- mixed precision helpers (FP64 side)
// r = b - v (FP64) and rr = (r, r), bb = (b, b)
__global__ __launch_bounds__(256) void k_res64(int64_t n, const double* __restrict__ b,
                                               const double* __restrict__ v, double* __restrict__ r,
                                               double* part, Scal* S) {
  double acc[2] = {0.0, 0.0};
  for (int64_t i = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kRedThreads) {
    const double ri = b[i] - v[i];
    r[i] = ri;
    acc[0] += ri * ri;
    acc[1] += b[i] * b[i];
  }
  double tot[2];
  if (finish_reduction<2>(acc, part, S, tot) && threadIdx.x == 0) {
    S->rr = tot[0];
    S->bb = tot[1];
  }
}

// x += scale * d (FP64 accumulation of a partial solution of either precision)
template <class T>
__global__ void k_addT(int64_t n, double* __restrict__ x, const T* __restrict__ d, double scale) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] += scale * (double)d[i];
}

// out = (T)(r * inv), d = 0
template <class T, class TX>
__global__ void k_scaleT(int64_t n, const double* __restrict__ r, double inv, T* __restrict__ out,
                         TX* __restrict__ d) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    out[i] = (T)(r[i] * inv);
    d[i] = TX(0);
  }
}


// Flags a breakdown of the recurrence (the test hook below).
__global__ void k_force_breakdown(Scal* S) {
  if (threadIdx.x == 0 && !S->done) {
    S->breakdown = 1;
    S->done = 1;
  }
}

__global__ void k_set_it(Scal* S, int it) {
  if (threadIdx.x == 0) S->it = it;
}

__global__ void k_zero_scal(Scal* S) {
  if (threadIdx.x == 0) {
    S->it = 0;
    S->done = 0;
    S->breakdown = 0;
    S->counter = 0;
  }
}

// ---- GMRES helpers (FP64)
// part[j][blk] = partial of (V_j, w) for j < nv (grid: blocks x nv)
__global__ __launch_bounds__(256) void k_gm_dots(int64_t n, const double* __restrict__ V,
                                                 int64_t ldv, const double* __restrict__ w,
                                                 double* part) {
  __shared__ double sh[256];
  const int j = blockIdx.y;
  const double* vj = V + (int64_t)j * ldv;
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    acc += vj[i] * w[i];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(int64_t)j * gridDim.x + blockIdx.x] = sh[0];
}

__global__ void k_gm_sum(const double* part, int np, double* out) {
  __shared__ double sh[256];
  const int j = blockIdx.x;
  double acc = 0.0;
  for (int i = threadIdx.x; i < np; i += 256) acc += part[(int64_t)j * np + i];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[j] = sh[0];
}

// w += sign * sum_j c_j V_j
__global__ void k_gm_comb(int64_t n, const double* __restrict__ V, int64_t ldv, int nv,
                          const double* __restrict__ c, double sign, double* __restrict__ w) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int j = 0; j < nv; ++j) acc += c[j] * V[(int64_t)j * ldv + i];
    w[i] += sign * acc;
  }
}

__global__ void k_gm_scale(int64_t n, const double* __restrict__ w, double a, double* __restrict__ v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    v[i] = a * w[i];
}

__global__ void k_gm_res(int64_t n, const double* __restrict__ b, const double* __restrict__ v,
                         double* __restrict__ r) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    r[i] = b[i] - v[i];
}

// ================================================================== host
namespace {

using Clock = std::chrono::steady_clock;

// Test hook for the breakdown restart: CPM_TEST_BREAKDOWN_AT=k makes an FP64
// BiCGSTAB solve flag a breakdown once (rho = (rh, r) treated as zero) at its
// first convergence check after k iterations, so that the restart from the
// current iterate with a new shadow residual runs on demand.  Read per solve.
int test_breakdown_at() {
  const char* e = std::getenv("CPM_TEST_BREAKDOWN_AT");
  return e && e[0] ? std::atoi(e) : -1;
}

// CPM_TRACE=1 prints the refinement history to stderr.
bool trace_on() {
  static const int on = [] {
    const char* e = std::getenv("CPM_TRACE");
    return e && e[0] && e[0] != '0' ? 1 : 0;
  }();
  return on != 0;
}

struct Pinned {
  Scal* h = nullptr;
  Pinned() { CPM_HIP(hipHostMalloc((void**)&h, sizeof(Scal), hipHostMallocDefault)); }
  ~Pinned() { if (h) (void)hipHostFree(h); }
};

// BiCGSTAB on one right-hand side.  Vectors are band scratch slots.  The
// recurrence vectors are of type T; the iterate passed to iteration() and
// solve() is of type TX (TX = double with T = float: the FP32 recurrence
// accumulates its solution in FP64).
template <class T, class TX = T>
struct Bicg {
  const cpm_band* b;
  hipStream_t st;
  int64_t n;
  double m, nn, gamma;
  bool transpose;
  T *r, *rh, *p, *v, *s, *t;
  double* part;
  double* dpart;   // partials of the dot products fused into the applies
  int dnp, fin_g;
  Scal* S;
  Pinned pin;
  int ew_grid, red_g;
  hipGraphExec_t gexec = nullptr;
  int graph_iters = 0;
  TX* gx_x = nullptr;

  Bicg(const cpm_band* b_, hipStream_t st_, double m_, double n_, double gamma_, bool tr, int slot0)
      : b(b_), st(st_), n(b_->n), m(m_), nn(n_), gamma(gamma_), transpose(tr) {
    const size_t vb = sizeof(T) * (size_t)n;
    r = (T*)band_scratch(b, slot0 + 0, vb);
    rh = (T*)band_scratch(b, slot0 + 1, vb);
    p = (T*)band_scratch(b, slot0 + 2, vb);
    v = (T*)band_scratch(b, slot0 + 3, vb);
    s = (T*)band_scratch(b, slot0 + 4, vb);
    t = (T*)band_scratch(b, slot0 + 5, vb);
    part = (double*)band_scratch(b, slot0 + 6, sizeof(double) * 2 * kMaxParts);
    S = (Scal*)band_scratch(b, slot0 + 7, sizeof(Scal));
    dnp = apply_dot_parts(b, tr, sizeof(T) == 4);
    dpart = (double*)band_scratch(b, slot0 + 8, sizeof(double) * 2 * (size_t)dnp);
    fin_g = (int)std::max<int64_t>(1, std::min<int64_t>(256, (dnp + 1023) / 1024));
    CPM_HIP(hipMemsetAsync(S, 0, sizeof(Scal), st));
    ew_grid = grid_for(n, 256, 4096);
    red_g = red_grid(n);
    // make sure every scratch buffer exists before any graph capture
    band_scratch(b, 0, apply_scratch_bytes(b, 1));
    if (gamma != 0.0) {
      band_scratch(b, 3, sizeof(double) * 256 + 64);
      band_scratch(b, 4, sizeof(double) + 64);
    }
    if (transpose) {
      band_scratch(b, 1, sizeof(double) * (size_t)n);
      band_scratch(b, 2, sizeof(double) * (size_t)n);
    }
  }
  ~Bicg() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
  }

  // out = A in; with dy, also the partials of (dy, out) and (out, out)
  void apply(const T* in, T* out, const T* dy = nullptr) {
    double* dp = dy ? dpart : nullptr;
    if (transpose) apply_transpose_impl<T>(b, m, nn, 1, in, out, st, nullptr, gamma, dy, dp);
    else apply_impl<T>(b, m, nn, 1, in, out, st, nullptr, gamma, dy, dp);
  }

  // r = rhs - A x, rh = p = r, v = 0, beta = 0 (so the first direction
  // update of an iteration leaves p = r); x is read only when x_zero is false,
  // which needs TX = T
  void init(const T* rhs, const TX* x, bool x_zero, double tol) {
    if (!x_zero) {
      if constexpr (std::is_same<T, TX>::value) apply(x, v);
      else CPM_FAIL(CPM_E_INVALID, "internal: warm start of a mixed-type recurrence");
    }
    hipLaunchKernelGGL(k_init<T>, dim3(red_g), dim3(kRedThreads), 0, st, n, rhs, v, !x_zero, r,
                       rh, p, part, S, tol);
    hipLaunchKernelGGL(k_zero<T>, dim3(ew_grid), dim3(256), 0, st, n, v);
    CPM_LAUNCH_CHECK();
  }

  // One BiCGSTAB step, starting with the direction update so that a step
  // ends right after the new residual (where an update can take place).
  void iteration(TX* x) {
    hipLaunchKernelGGL(k_p<T>, dim3(ew_grid), dim3(256), 0, st, n, r, p, v, S);
    apply(p, v, rh);
    hipLaunchKernelGGL(k_dot_fin<0>, dim3(fin_g), dim3(kRedThreads), 0, st, dpart, dnp, part, S);
    hipLaunchKernelGGL(k_s<T>, dim3(ew_grid), dim3(256), 0, st, n, r, v, s, S);
    apply(s, t, s);
    hipLaunchKernelGGL(k_dot_fin<1>, dim3(fin_g), dim3(kRedThreads), 0, st, dpart, dnp, part, S);
    hipLaunchKernelGGL((k_xr<T, TX>), dim3(red_g), dim3(kRedThreads), 0, st, n, x, p, s, t, r, rh,
                       part, S);
    CPM_LAUNCH_CHECK();
  }

  void run_iters(TX* x, int k, bool use_graph) {
    if (!use_graph) {
      for (int i = 0; i < k; ++i) iteration(x);
      return;
    }
    if (!gexec || graph_iters != k || gx_x != x) {
      if (gexec) CPM_HIP(hipGraphExecDestroy(gexec));
      gexec = nullptr;
      hipGraph_t g;
      CPM_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
      try {
        for (int i = 0; i < k; ++i) iteration(x);
      } catch (...) {
        // end the capture and drop what it recorded before passing the error on
        hipGraph_t part = nullptr;
        if (hipStreamEndCapture(st, &part) == hipSuccess && part) (void)hipGraphDestroy(part);
        throw;
      }
      CPM_HIP(hipStreamEndCapture(st, &g));
      const hipError_t e = hipGraphInstantiate(&gexec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      CPM_HIP(e);
      graph_iters = k;
      gx_x = x;
    }
    CPM_HIP(hipGraphLaunch(gexec, st));
  }

  const Scal& read() {
    CPM_HIP(hipMemcpyAsync(pin.h, S, sizeof(Scal), hipMemcpyDeviceToHost, st));
    CPM_HIP(hipStreamSynchronize(st));
    return *pin.h;
  }

  // Solve A x = rhs to the recursive residual tol (relative).  Returns the
  // iterations spent; breakdowns restart from the current iterate.
  int solve(const T* rhs, TX* x, bool x_zero, double tol, int maxit, int check_every,
            bool use_graph, int* restarts) {
    hipLaunchKernelGGL(k_zero_scal, dim3(1), dim3(64), 0, st, S);
    init(rhs, x, x_zero, tol);
    int it = 0;
    const int force_at = test_breakdown_at();
    bool forced = false;
    const Scal* h = &read();
    while (!h->done && it < maxit) {
      const int k = std::min(check_every, maxit - it);
      run_iters(x, k, use_graph && k == check_every);
      h = &read();
      it = h->it;
      if (force_at >= 0 && !forced && !h->done && it >= force_at) {
        forced = true;
        hipLaunchKernelGGL(k_force_breakdown, dim3(1), dim3(64), 0, st, S);
        CPM_LAUNCH_CHECK();
        h = &read();
      }
      if (h->done && h->breakdown && !(h->rr <= h->tol2)) {
        if (++*restarts > 50) break;
        const int keep = h->it;
        hipLaunchKernelGGL(k_zero_scal, dim3(1), dim3(64), 0, st, S);
        init(rhs, x, false, tol);
        hipLaunchKernelGGL(k_set_it, dim3(1), dim3(64), 0, st, S, keep);
        CPM_LAUNCH_CHECK();
        h = &read();
      }
    }
    return h->it;
  }
};

// one FP64 apply into v and the FP64 residual; returns ||b - A x||, ||b||
std::pair<double, double> residual64(const cpm_band* b, hipStream_t st, double m, double nn,
                                     double gamma, bool tr, const double* rhs, const double* x,
                                     double* r, double* v, double* part, Scal* S, Pinned& pin) {
  if (tr) apply_transpose_impl<double>(b, m, nn, 1, x, v, st, nullptr, gamma);
  else apply_impl<double>(b, m, nn, 1, x, v, st, nullptr, gamma);
  hipLaunchKernelGGL(k_res64, dim3(red_grid(b->n)), dim3(kRedThreads), 0, st, b->n, rhs, v, r,
                     part, S);
  CPM_LAUNCH_CHECK();
  CPM_HIP(hipMemcpyAsync(pin.h, S, sizeof(Scal), hipMemcpyDeviceToHost, st));
  CPM_HIP(hipStreamSynchronize(st));
  return {std::sqrt(pin.h->rr), std::sqrt(pin.h->bb)};
}

// GMRES(k): Arnoldi with classical Gram-Schmidt and one re-orthogonalisation
// on the device, Givens rotations of the Hessenberg on the host (one read
// back per iteration; meant for small systems such as curves in R^2).
void gmres64(const cpm_band* b, const cpm_solve_opts& o, const double* rhs, double* x,
             cpm_solve_stats& stt, hipStream_t st, bool tr) {
  const int64_t n = b->n;
  const int k = std::min(200, o.restart > 0 ? o.restart : 50);
  const int maxit = o.maxit > 0 ? o.maxit : 20000;
  const double tol = o.tol > 0 ? o.tol : 1e-8;
  double* V = (double*)band_scratch(b, 70, sizeof(double) * (size_t)n * (k + 1));
  double* w = (double*)band_scratch(b, 71, sizeof(double) * n);
  const int gd = (int)std::min<int64_t>(256, (n + 255) / 256);
  double* part = (double*)band_scratch(b, 72, sizeof(double) * (size_t)gd * (k + 1));
  double* dv = (double*)band_scratch(b, 73, sizeof(double) * (k + 2));
  double* hp = nullptr;
  CPM_HIP(hipHostMalloc((void**)&hp, sizeof(double) * (k + 2), hipHostMallocDefault));
  struct HF { double* p; ~HF() { if (p) (void)hipHostFree(p); } } hf{hp};
  auto A = [&](const double* in, double* out) {
    if (tr) apply_transpose_impl<double>(b, o.m, o.n, 1, in, out, st, nullptr, o.gauge);
    else apply_impl<double>(b, o.m, o.n, 1, in, out, st, nullptr, o.gauge);
  };
  const int eg = grid_for(n, 256, 4096);
  auto dots = [&](int nv, const double* vec) {   // dv[0..nv) = (V_j, vec)
    hipLaunchKernelGGL(k_gm_dots, dim3(gd, nv), dim3(256), 0, st, n, V, n, vec, part);
    hipLaunchKernelGGL(k_gm_sum, dim3(nv), dim3(256), 0, st, part, gd, dv);
    CPM_LAUNCH_CHECK();
    CPM_HIP(hipMemcpyAsync(hp, dv, sizeof(double) * nv, hipMemcpyDeviceToHost, st));
    CPM_HIP(hipStreamSynchronize(st));
  };
  auto norm_of = [&](const double* vec) {        // ||vec|| via V_0 slot trick
    hipLaunchKernelGGL(k_gm_dots, dim3(gd, 1), dim3(256), 0, st, n, vec, n, vec, part);
    hipLaunchKernelGGL(k_gm_sum, dim3(1), dim3(256), 0, st, part, gd, dv);
    CPM_LAUNCH_CHECK();
    CPM_HIP(hipMemcpyAsync(hp, dv, sizeof(double), hipMemcpyDeviceToHost, st));
    CPM_HIP(hipStreamSynchronize(st));
    return std::sqrt(hp[0]);
  };
  const double bn = norm_of(rhs);
  if (bn == 0.0) {
    CPM_HIP(hipMemsetAsync(x, 0, sizeof(double) * n, st));
    stt.converged = 1;
    stt.relres = 0.0;
    return;
  }
  std::vector<double> H((size_t)(k + 1) * k), cs(k), sn(k), g(k + 1), y(k);
  int its = 0;
  double rel = 1.0;
  while (its < maxit) {
    A(x, w);
    hipLaunchKernelGGL(k_gm_res, dim3(eg), dim3(256), 0, st, n, rhs, w, w);
    CPM_LAUNCH_CHECK();
    const double beta = norm_of(w);
    rel = beta / bn;
    stt.relres = rel;
    ++stt.outer_iters;
    if (rel <= tol) break;
    hipLaunchKernelGGL(k_gm_scale, dim3(eg), dim3(256), 0, st, n, w, 1.0 / beta, V);
    std::fill(H.begin(), H.end(), 0.0);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int j = 0;
    for (; j < k && its < maxit; ++j) {
      A(V + (int64_t)j * n, w);
      // two passes of classical Gram-Schmidt
      for (int pass = 0; pass < 2; ++pass) {
        dots(j + 1, w);
        for (int i = 0; i <= j; ++i) H[(size_t)i * k + j] += hp[i];
        CPM_HIP(hipMemcpyAsync(dv, hp, sizeof(double) * (j + 1), hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(k_gm_comb, dim3(eg), dim3(256), 0, st, n, V, n, j + 1, dv, -1.0, w);
        CPM_LAUNCH_CHECK();
      }
      const double hn = norm_of(w);
      H[(size_t)(j + 1) * k + j] = hn;
      if (hn > 0.0)
        hipLaunchKernelGGL(k_gm_scale, dim3(eg), dim3(256), 0, st, n, w, 1.0 / hn,
                           V + (int64_t)(j + 1) * n);
      for (int i = 0; i < j; ++i) {
        const double a = H[(size_t)i * k + j], c2 = H[(size_t)(i + 1) * k + j];
        H[(size_t)i * k + j] = cs[i] * a + sn[i] * c2;
        H[(size_t)(i + 1) * k + j] = -sn[i] * a + cs[i] * c2;
      }
      const double a = H[(size_t)j * k + j], c2 = H[(size_t)(j + 1) * k + j];
      const double den = std::hypot(a, c2);
      cs[j] = den > 0 ? a / den : 1.0;
      sn[j] = den > 0 ? c2 / den : 0.0;
      H[(size_t)j * k + j] = den;
      H[(size_t)(j + 1) * k + j] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      ++its;
      if (std::fabs(g[j + 1]) <= tol * bn || hn == 0.0) {
        ++j;
        break;
      }
    }
    // back substitution and x += V y
    for (int i = j - 1; i >= 0; --i) {
      double s2 = g[i];
      for (int q = i + 1; q < j; ++q) s2 -= H[(size_t)i * k + q] * y[q];
      y[i] = s2 / H[(size_t)i * k + i];
    }
    CPM_HIP(hipMemcpyAsync(dv, y.data(), sizeof(double) * j, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_gm_comb, dim3(eg), dim3(256), 0, st, n, V, n, j, dv, 1.0, x);
    CPM_LAUNCH_CHECK();
    CPM_HIP(hipStreamSynchronize(st));
  }
  stt.krylov_iters += its;
  stt.converged = rel <= tol ? 1 : 0;
}

// Shared state of a reliable-update solve of A x = rhs: the recurrence runs
// on A d = r0 / sigma; x accumulates sigma d in FP64.
struct RU {
  const cpm_band* b;
  hipStream_t st;
  double m, nn, gamma;
  bool tr;
  const double* rhs;
  double* x;
  double *r64, *v64, *part;
  Scal* S;
  Pinned* pin;
  double bn, sigma, delta, tol;
  int maxit, ce;
  bool graph;
  cpm_solve_stats* stt;
  int its = 0;

  std::pair<double, double> residual() {
    return residual64(b, st, m, nn, gamma, tr, rhs, x, r64, v64, part, S, *pin);
  }
};

enum { RU_CONVERGED = 0, RU_STALLED = 1, RU_MAXIT = 2 };

// Runs a recurrence of precision T with reliable updates until the FP64
// residual reaches tol.  The recurrence solves A d = r / sigma and keeps its
// partial solution d in TX (FP64 for the mixed solve).  An update happens
// when the recursive residual has dropped by delta since the last one, when
// the recurrence stops (converged or broken down), when its residual has
// grown kBlowup-fold over the last true one, or after max_cycle iterations
// without any of these.  It adds sigma d into x and recomputes r = b - A x in
// FP64, then starts the recurrence afresh from the true residual with it as
// the new shadow residual (r_hat = r, d = 0), as Eigen's BiCGSTAB restarts
// when rho vanishes.  Restarting at every update, rather than substituting
// the true residual into the running recurrence, measured fewer iterations
// in FP32 (1,048 against 1,434 on the sphere with a latitude boundary at
// h = 1/256, 3,840 against 6,492 on the torus at h = 1/512): an FP32
// recurrence loses its bi-orthogonality to the old shadow residual.  An
// update that raised the FP64 residual is taken back, so x is always the
// best iterate.  The run ends (RU_STALLED) when an update follows a
// breakdown or growth, or fails to halve the FP64 residual, more than
// max_restarts times.
constexpr double kBlowup = 1e3;

template <class T, class TX>
int ru_run(RU& c, Bicg<T, TX>& k, TX* d, T* rT, double rn, int max_cycle, int max_restarts) {
  const int64_t n = c.b->n;
  const double inv = 1.0 / c.sigma;
  const int eg = grid_for(n, 256, 4096);
  double maxr = rn * inv, base = maxr, prev = rn;
  int last = k.read().it, cycle0 = last, failures = 0;
  while (c.its < c.maxit) {
    const int kk = std::min(c.ce, c.maxit - c.its);
    k.run_iters(d, kk, c.graph && kk == c.ce);
    const Scal& h = k.read();
    c.its += h.it - last;
    last = h.it;
    const double rrec = std::sqrt(h.rr);
    const bool bad = !std::isfinite(h.rr);
    const bool blowup = !bad && rrec > kBlowup * base;
    if (!bad) maxr = std::max(maxr, rrec);
    const bool forced = h.it - cycle0 >= max_cycle;
    if (!(h.done || bad || blowup || rrec < c.delta * maxr || forced)) continue;
    const bool broken = h.breakdown || bad || blowup;
    if (!bad) {   // a non-finite recursion leaves x as it was at the last update
      hipLaunchKernelGGL(k_addT<TX>, dim3(eg), dim3(256), 0, c.st, n, c.x, d, c.sigma);
      CPM_LAUNCH_CHECK();
    }
    rn = c.residual().first;
    c.stt->relres = rn / c.bn;
    ++c.stt->outer_iters;
    if (trace_on())
      std::fprintf(stderr, "[cpm] %s update %d: recursive %.3e true relres %.3e its %d%s%s%s\n",
                   sizeof(T) == 4 ? "FP32" : "FP64", c.stt->outer_iters, rrec * c.sigma / c.bn,
                   c.stt->relres, c.its, h.breakdown ? " (breakdown)" : "",
                   blowup || bad ? " (growth)" : "", forced ? " (forced)" : "");
    if (c.stt->relres <= c.tol) return RU_CONVERGED;
    if (!std::isfinite(rn) || !(rn <= prev)) {
      if (!bad) {   // take the update back
        hipLaunchKernelGGL(k_addT<TX>, dim3(eg), dim3(256), 0, c.st, n, c.x, d, -c.sigma);
        CPM_LAUNCH_CHECK();
      }
      rn = c.residual().first;   // r64 holds the residual of x again
      c.stt->relres = rn / c.bn;
    }
    if (broken || !(rn < 0.5 * prev)) {
      if (++failures > max_restarts) return RU_STALLED;
      ++c.stt->restarts;
    }
    prev = std::min(prev, rn);
    hipLaunchKernelGGL((k_scaleT<T, TX>), dim3(eg), dim3(256), 0, c.st, n, c.r64, inv, rT, d);
    hipLaunchKernelGGL(k_zero_scal, dim3(1), dim3(64), 0, c.st, k.S);
    CPM_LAUNCH_CHECK();
    k.init(rT, nullptr, true, 0.5 * c.tol * c.bn / rn);
    last = cycle0 = 0;
    maxr = base = rn * inv;
  }
  return RU_MAXIT;
}

void solve_one(const cpm_band* b, const cpm_solve_opts& o, const double* rhs, double* x,
               cpm_solve_stats& stt, hipStream_t st, bool tr) {
  const int64_t n = b->n;
  {
    // non-finite data would only surface as a failed convergence; refuse it
    double* r64 = (double*)band_scratch(b, 20, sizeof(double) * n);
    double* v64 = (double*)band_scratch(b, 21, sizeof(double) * n);
    double* part = (double*)band_scratch(b, 22, sizeof(double) * 2 * kMaxParts);
    Scal* S = (Scal*)band_scratch(b, 23, sizeof(Scal));
    CPM_HIP(hipMemsetAsync(S, 0, sizeof(Scal), st));
    Pinned pin;
    auto rb = residual64(b, st, o.m, o.n, o.gauge, tr, rhs, x, r64, v64, part, S, pin);
    if (!std::isfinite(rb.second))
      CPM_FAIL(CPM_E_INVALID, "the right-hand side holds non-finite values");
    if (!std::isfinite(rb.first))
      CPM_FAIL(CPM_E_INVALID, "the initial guess holds non-finite values");
  }
  if (o.mode == CPM_SOLVE_GMRES) {
    gmres64(b, o, rhs, x, stt, st, tr);
    return;
  }
  const int maxit = o.maxit > 0 ? o.maxit : 20000;
  const int ce = o.check_every > 0 ? o.check_every : 16;
  const double tol = o.tol > 0 ? o.tol : 1e-8;
  const double gamma = o.gauge;
  const bool graph = o.use_graph != 0;
  double* r64 = (double*)band_scratch(b, 20, sizeof(double) * n);
  double* v64 = (double*)band_scratch(b, 21, sizeof(double) * n);
  double* part = (double*)band_scratch(b, 22, sizeof(double) * 2 * kMaxParts);
  Scal* S = (Scal*)band_scratch(b, 23, sizeof(Scal));
  CPM_HIP(hipMemsetAsync(S, 0, sizeof(Scal), st));
  Pinned pin;
  int its = 0, restarts = 0;
  // Plain FP64 BiCGSTAB, restarted from the current x while the recursive
  // residual has drifted from the true one.  The iterate of smallest true
  // residual is kept, so a pass cut short by maxit never returns a worse one.
  auto plain64 = [&](double tol_) {
    Bicg<double> k(b, st, o.m, o.n, gamma, tr, 30);
    double* xbest = nullptr;
    double best = HUGE_VAL;
    for (int rep = 0; rep < 20 && its < maxit; ++rep) {
      its += k.solve(rhs, x, false, tol_, maxit - its, ce, graph, &restarts);
      auto rb = residual64(b, st, o.m, o.n, gamma, tr, rhs, x, r64, v64, part, S, pin);
      stt.relres = rb.second > 0 ? rb.first / rb.second : 0.0;
      ++stt.outer_iters;
      if (trace_on())
        std::fprintf(stderr, "[cpm] f64 pass %d relres %.3e iterations %d restarts %d\n", rep,
                     stt.relres, its, restarts);
      if (stt.relres <= tol) return true;
      if (stt.relres < best) {
        if (!xbest) xbest = (double*)band_scratch(b, 28, sizeof(double) * n);
        CPM_HIP(hipMemcpyAsync(xbest, x, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
        best = stt.relres;
      }
    }
    if (xbest && !(stt.relres <= best)) {
      CPM_HIP(hipMemcpyAsync(x, xbest, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
      stt.relres = best;
    }
    return false;
  };
  // Mixed precision: one FP32 BiCGSTAB recurrence on A d = r0 / sigma with
  // reliable updates (ru_run).  The recurrence vectors are FP32; the FP32
  // apply computes in FP64 (FP64 weights and intermediate vectors), so it
  // differs from the FP64 operator only by the rounding of the stored
  // interpolation fractions; the partial solution d is accumulated in FP64
  // and convergence is decided on the FP64 residual only.  If the updates
  // stop making progress, the solve continues with FP64 BiCGSTAB from the
  // refined x.
  auto mixed_ru = [&]() {
    RU c{b, st, o.m, o.n, gamma, tr, rhs, x, r64, v64, part, S, &pin};
    auto rb = c.residual();
    c.bn = rb.second;
    const double rn = rb.first;
    stt.relres = c.bn > 0 ? rn / c.bn : 0.0;
    if (c.bn == 0.0 || stt.relres <= tol) return true;
    if (!__builtin_isfinite(rn)) return false;
    c.sigma = rn;
    c.delta = o.inner_tol > 0 ? o.inner_tol : 0.1;
    c.tol = tol;
    c.maxit = maxit;
    c.ce = ce;
    c.graph = graph;
    c.stt = &stt;
    const double inv = 1.0 / c.sigma;
    Bicg<float, double> k32(b, st, o.m, o.n, gamma, tr, 10);
    float* r32 = (float*)band_scratch(b, 24, sizeof(float) * n);
    double* d64 = (double*)band_scratch(b, 25, sizeof(double) * n);
    hipLaunchKernelGGL((k_scaleT<float, double>), dim3(grid_for(n, 256, 4096)), dim3(256), 0, st,
                       n, r64, inv, r32, d64);
    hipLaunchKernelGGL(k_zero_scal, dim3(1), dim3(64), 0, st, k32.S);
    CPM_LAUNCH_CHECK();
    k32.init(r32, nullptr, true, 0.5 * tol * c.bn * inv);
    const int status = ru_run<float, double>(c, k32, d64, r32, rn, 1000, 4);
    its += c.its;
    if (status == RU_CONVERGED) return true;
    if (status == RU_MAXIT) return false;
    stt.fallback_f64 = 1;
    return plain64(tol);
  };
  bool ok = false;
  if (o.mode == CPM_SOLVE_F64) {
    ok = plain64(tol);
  } else {
    ok = mixed_ru();
  }
  stt.krylov_iters += its;
  stt.restarts += restarts;
  stt.converged = ok ? 1 : 0;
}

cpm_status solve_entry(const cpm_band* b, const cpm_solve_opts* o, int nrhs, const double* rhs,
                       double* x, cpm_solve_stats* stats, void* hip_stream, bool tr) {
  cpm_status ret = CPM_OK;
  cpm_status g = guard([&] {
    if (!b || !o || !rhs || !x || nrhs < 1) CPM_FAIL(CPM_E_INVALID, "bad argument");
    if (o->mode != CPM_SOLVE_MIXED && o->mode != CPM_SOLVE_F64 && o->mode != CPM_SOLVE_GMRES)
      CPM_FAIL(CPM_E_INVALID, "unknown solve mode %d", o->mode);
    if (tr && o->gauge != 0.0) CPM_FAIL(CPM_E_INVALID, "the gauge is not supported for the adjoint");
    const auto t0 = Clock::now();
    hipStream_t caller = (hipStream_t)hip_stream;
    // the solve is host-synchronous; it runs on a private stream so that its
    // iterations can be captured into a graph even when the caller passes the
    // null stream
    CPM_HIP(hipStreamSynchronize(caller));
    hipStream_t st = nullptr;
    CPM_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    struct StreamGuard {
      hipStream_t s;
      ~StreamGuard() { (void)hipStreamSynchronize(s); (void)hipStreamDestroy(s); }
    } sg{st};
    cpm_solve_stats agg{};
    agg.converged = 1;
    double worst = 0.0;
    for (int r = 0; r < nrhs; ++r) {
      cpm_solve_stats s1{};
      solve_one(b, *o, rhs + (int64_t)r * b->n, x + (int64_t)r * b->n, s1, st, tr);
      agg.converged &= s1.converged;
      agg.outer_iters += s1.outer_iters;
      agg.krylov_iters += s1.krylov_iters;
      agg.restarts += s1.restarts;
      agg.fallback_f64 |= s1.fallback_f64;
      worst = std::max(worst, s1.relres);
    }
    agg.relres = worst;
    CPM_HIP(hipStreamSynchronize(st));
    agg.time_ms = std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
    if (stats) *stats = agg;
    if (!agg.converged) {
      set_error("solve did not reach tol %.3g: relative residual %.3g after %d iterations",
                o->tol, worst, agg.krylov_iters);
      ret = CPM_E_NOCONV;
    }
  });
  return g != CPM_OK ? g : ret;
}

}  // namespace
}  // namespace cpm

using namespace cpm;

extern "C" cpm_status cpm_solve(const cpm_band* b, const cpm_solve_opts* o, int nrhs,
                                const double* rhs, double* x, cpm_solve_stats* stats,
                                void* hip_stream) {
  return solve_entry(b, o, nrhs, rhs, x, stats, hip_stream, false);
}

extern "C" cpm_status cpm_solve_adjoint(const cpm_band* b, const cpm_solve_opts* o, int nrhs,
                                        const double* rhs, double* lambda,
                                        cpm_solve_stats* stats, void* hip_stream) {
  return solve_entry(b, o, nrhs, rhs, lambda, stats, hip_stream, true);
}

// Crank-Nicolson steps of u_t = Delta_S u with interior boundary conditions
// (the heat test of Sec. 6.2; trapezoidal rule):
//   (I - dt/2 M) u^{k+1} = (I + dt/2 M) u^k + dt/2 (L - D)(e(g^k) + e(g^{k+1})).
// Each step solves with the given options, warm-started from u^k.
extern "C" cpm_status cpm_heat_cn(const cpm_band* b, double dt, int nsteps, const double* g,
                                  double* u, const cpm_solve_opts* o, cpm_solve_stats* stats,
                                  void* hip_stream) {
  cpm_status ret = CPM_OK;
  const cpm_status gs = guard([&] {
    if (!b || !u || !o) CPM_FAIL(CPM_E_INVALID, "null argument");
    if (!(dt > 0.0) || nsteps < 0) CPM_FAIL(CPM_E_INVALID, "dt must be > 0 and nsteps >= 0");
    if (o->mode != CPM_SOLVE_MIXED && o->mode != CPM_SOLVE_F64 && o->mode != CPM_SOLVE_GMRES)
      CPM_FAIL(CPM_E_INVALID, "unknown solve mode %d", o->mode);
    if (o->gauge != 0.0) CPM_FAIL(CPM_E_INVALID, "the gauge does not apply to time stepping");
    if (b->composite) CPM_FAIL(CPM_E_INVALID, "time stepping takes a single band");
    const auto t0 = Clock::now();
    CPM_HIP(hipStreamSynchronize((hipStream_t)hip_stream));
    hipStream_t st = nullptr;
    CPM_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    struct StreamGuard {
      hipStream_t s;
      ~StreamGuard() { (void)hipStreamSynchronize(s); (void)hipStreamDestroy(s); }
    } sg{st};
    double* rhs = (double*)band_scratch(b, 80, sizeof(double) * (size_t)b->n);
    cpm_solve_opts oo = *o;
    oo.m = 1.0;
    oo.n = -0.5 * dt;
    cpm_solve_stats agg{};
    agg.converged = 1;
    for (int k = 0; k < nsteps; ++k) {
      apply_impl<double>(b, 1.0, 0.5 * dt, 1, u, rhs, st);
      if (g && b->n_c) {
        add_dirichlet_term(b, -0.5 * dt, g + (int64_t)k * b->n_c, 1, rhs, st);
        add_dirichlet_term(b, -0.5 * dt, g + (int64_t)(k + 1) * b->n_c, 1, rhs, st);
      }
      cpm_solve_stats s1{};
      solve_one(b, oo, rhs, u, s1, st, false);
      agg.outer_iters += s1.outer_iters;
      agg.krylov_iters += s1.krylov_iters;
      agg.restarts += s1.restarts;
      agg.fallback_f64 |= s1.fallback_f64;
      agg.relres = std::max(agg.relres, s1.relres);
      if (!s1.converged) {
        agg.converged = 0;
        set_error("time step %d did not reach tol %.3g (relative residual %.3g)", k, o->tol,
                  s1.relres);
        ret = CPM_E_NOCONV;
        break;
      }
    }
    CPM_HIP(hipStreamSynchronize(st));
    agg.time_ms = std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
    if (stats) *stats = agg;
  });
  return gs != CPM_OK ? gs : ret;
}
