// Batched solves: several bands (instances of uneven size, each with nrhs
// right-hand sides) solved together, one launch per kernel.
//
// The instances' device arrays are concatenated into one composite band
// (DOFs of instance i at [D_i, D_i + n_i)); the apply kernels run unchanged
// on it, with per-instance FD coefficients looked up through the instance id
// stored in each block's metadata.  The Krylov solver is BiCGSTAB with one
// set of scalars and one convergence flag per system (instance, right-hand
// side): every reduction is segmented over fixed chunks of one system, and
// the last workgroup of a system finishes that system's sums in a fixed
// order.  Mixed precision works as for one band: FP32 BiCGSTAB for the
// correction inside FP64 iterative refinement, per system.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <memory>

#include "cpm_internal.hpp"

namespace cpm {

struct BScal {
  double rho, rho_old, alpha, omega, beta;
  double bb, rr, tol2;
  int done, breakdown, it, active;
  unsigned counter;
  unsigned pad;
};

constexpr int kChunk = 32768;  // elements per reduction workgroup (256 x 128)
constexpr int kBT = 256;

// ---------------------------------------------------------------- concat
__global__ void k_cat_meta(const QMeta* in, QMeta* out, int64_t cnt, int add, int face_inst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cnt) return;
  QMeta q = in[i];
  if (face_inst >= 0 && (i & 7) == 7) {
    q.pad = face_inst;   // block metadata: instance id in entry 7
  } else {
    q.off += add;
  }
  out[i] = q;
}

__global__ void k_cat_int(const int* in, int* out, int64_t cnt, int add) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cnt) return;
  const int v = in[i];
  out[i] = v >= 0 ? v + add : v;
}

__global__ void k_fill_int(int* out, int64_t cnt, int val) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cnt) out[i] = val;
}

// ---------------------------------------------------------------- segmented
struct Seg {
  const int* csys;       // [nchunks] system of the chunk
  const int64_t* clo;    // [nchunks] first element
  const int64_t* chi;    // [nchunks] end
  const int* sfirst;     // [nsys] first chunk of the system
  const int* snch;       // [nsys] chunks of the system
};

template <int NR>
__device__ __forceinline__ void bwg_sum(double v[NR], double (*sh)[kBT]) {
  for (int k = 0; k < NR; ++k) sh[k][threadIdx.x] = v[k];
  __syncthreads();
  for (int o = kBT / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o)
      for (int k = 0; k < NR; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + o];
    __syncthreads();
  }
  for (int k = 0; k < NR; ++k) v[k] = sh[k][0];
}

// Partial sums of this chunk; true in the last workgroup of the system, with
// out[] the system's totals summed over its chunks in order.
template <int NR>
__device__ bool seg_finish(double v[NR], double* part, int nchunks, const Seg& g, int s,
                           BScal* S, double out[NR]) {
  __shared__ double sh[NR][kBT];
  __shared__ bool last;
  bwg_sum<NR>(v, sh);
  if (threadIdx.x == 0) {
    for (int k = 0; k < NR; ++k) part[(int64_t)k * nchunks + blockIdx.x] = v[k];
    __threadfence();
    const unsigned prev = atomicAdd(&S[s].counter, 1u);
    last = (int)prev == g.snch[s] - 1;
  }
  __syncthreads();
  if (!last) return false;
  __threadfence();
  double acc[NR];
  for (int k = 0; k < NR; ++k) acc[k] = 0.0;
  const int c0 = g.sfirst[s], nc = g.snch[s];
  for (int c = threadIdx.x; c < nc; c += kBT)
    for (int k = 0; k < NR; ++k)
      acc[k] += __builtin_nontemporal_load(&part[(int64_t)k * nchunks + c0 + c]);
  __syncthreads();
  bwg_sum<NR>(acc, sh);
  for (int k = 0; k < NR; ++k) out[k] = acc[k];
  if (threadIdx.x == 0) S[s].counter = 0;
  return true;
}

#define SEG_PROLOGUE                                  \
  const int s = g.csys[blockIdx.x];                   \
  const int64_t lo = g.clo[blockIdx.x], hi = g.chi[blockIdx.x]

template <class T>
__global__ __launch_bounds__(256) void k_binit(int nchunks, Seg g, const T* __restrict__ b,
                                               const T* __restrict__ v, int has_v, T* r, T* rh,
                                               T* p, double* part, BScal* S, double tol) {
  SEG_PROLOGUE;
  if (!S[s].active) return;
  double acc[2] = {0.0, 0.0};
  for (int64_t i = lo + threadIdx.x; i < hi; i += kBT) {
    const T ri = has_v ? b[i] - v[i] : b[i];
    r[i] = ri;
    rh[i] = ri;
    p[i] = ri;
    acc[0] += (double)ri * (double)ri;
    acc[1] += (double)b[i] * (double)b[i];
  }
  double tot[2];
  if (seg_finish<2>(acc, part, nchunks, g, s, S, tot) && threadIdx.x == 0) {
    BScal& q = S[s];
    q.rho = q.rho_old = q.rr = tot[0];
    q.bb = tot[1];
    q.tol2 = tol * tol * tot[1];
    q.alpha = q.omega = 1.0;
    q.beta = 0.0;
    q.breakdown = 0;
    q.done = tot[0] <= q.tol2 ? 1 : 0;
  }
}

template <class T>
__global__ __launch_bounds__(256) void k_bs(int nchunks, Seg g, const T* __restrict__ r,
                                            const T* __restrict__ v, T* __restrict__ sv,
                                            const BScal* S) {
  SEG_PROLOGUE;
  if (S[s].done) return;
  const T al = (T)S[s].alpha;
  for (int64_t i = lo + threadIdx.x; i < hi; i += kBT) sv[i] = r[i] - al * v[i];
}

// Finishes a dot product fused into the composite apply, one workgroup per
// system s = r * ninst + i: the partials of right-hand side r lie at dp + 2 r
// np (first value) and + np (second value); instance i owns the Laplacian
// pass's block partials [boff[i], boff[i + 1]) and the explicit rows'
// partials lp0 + [loff[i], loff[i + 1]).  Summed in a fixed order.  MODE 0:
// alpha = rho / (rh, v); MODE 1: omega = (t, s) / (t, t).
template <int MODE>
__global__ __launch_bounds__(256) void k_bdot_fin(int ninst, const double* __restrict__ dp,
                                                  int np, int lp0, const int* __restrict__ boff,
                                                  const int* __restrict__ loff, BScal* S) {
  __shared__ double sh[2][kBT];
  const int s = blockIdx.x, r = s / ninst, i = s % ninst;
  if (S[s].done) return;
  const double* d = dp + (size_t)2 * r * np;
  double v[2] = {0.0, 0.0};
  for (int k = boff[i] + threadIdx.x; k < boff[i + 1]; k += kBT) {
    v[0] += d[k];
    v[1] += d[np + k];
  }
  for (int k = lp0 + loff[i] + threadIdx.x; k < lp0 + loff[i + 1]; k += kBT) {
    v[0] += d[k];
    v[1] += d[np + k];
  }
  bwg_sum<2>(v, sh);
  if (threadIdx.x != 0) return;
  if (MODE == 0) {
    if (v[0] == 0.0 || !__builtin_isfinite(v[0])) {
      S[s].breakdown = 1;
      S[s].done = 1;
    } else {
      S[s].alpha = S[s].rho / v[0];
    }
  } else {
    S[s].omega = (v[1] == 0.0 || !__builtin_isfinite(v[1])) ? 0.0 : v[0] / v[1];
  }
}

template <class T, class TX>
__global__ __launch_bounds__(256) void k_bxr(int nchunks, Seg g, TX* __restrict__ x,
                                             const T* __restrict__ p, const T* __restrict__ sv,
                                             const T* __restrict__ t, T* __restrict__ r,
                                             const T* __restrict__ rh, double* part, BScal* S) {
  SEG_PROLOGUE;
  if (S[s].done) return;
  const T om = (T)S[s].omega;
  const TX alx = (TX)S[s].alpha, omx = (TX)S[s].omega;
  double acc[2] = {0.0, 0.0};
  for (int64_t i = lo + threadIdx.x; i < hi; i += kBT) {
    const T si = sv[i];
    x[i] = x[i] + alx * (TX)p[i] + omx * (TX)si;
    const T ri = si - om * t[i];
    r[i] = ri;
    acc[0] += (double)rh[i] * (double)ri;
    acc[1] += (double)ri * (double)ri;
  }
  double tot[2];
  if (seg_finish<2>(acc, part, nchunks, g, s, S, tot) && threadIdx.x == 0) {
    BScal& q = S[s];
    q.it += 1;
    q.rr = tot[1];
    if (!__builtin_isfinite(tot[1])) {
      q.breakdown = 1;
      q.done = 1;
    } else if (tot[1] <= q.tol2) {
      q.done = 1;
    } else if (tot[0] == 0.0 || q.omega == 0.0) {
      q.breakdown = 1;
      q.done = 1;
    } else {
      q.rho_old = q.rho;
      q.rho = tot[0];
      q.beta = (q.rho / q.rho_old) * (q.alpha / q.omega);
    }
  }
}

template <class T>
__global__ __launch_bounds__(256) void k_bp(int nchunks, Seg g, const T* __restrict__ r,
                                            T* __restrict__ p, const T* __restrict__ v,
                                            const BScal* S) {
  SEG_PROLOGUE;
  if (S[s].done) return;
  const T be = (T)S[s].beta, om = (T)S[s].omega;
  for (int64_t i = lo + threadIdx.x; i < hi; i += kBT) p[i] = r[i] + be * (p[i] - om * v[i]);
}

// FP64 residual r = b - v per system, with (r, r) and (b, b)
__global__ __launch_bounds__(256) void k_bres64(int nchunks, Seg g, const double* __restrict__ b,
                                                const double* __restrict__ v,
                                                double* __restrict__ r, double* part, BScal* S) {
  SEG_PROLOGUE;
  double acc[2] = {0.0, 0.0};
  for (int64_t i = lo + threadIdx.x; i < hi; i += kBT) {
    const double ri = b[i] - v[i];
    r[i] = ri;
    acc[0] += ri * ri;
    acc[1] += b[i] * b[i];
  }
  double tot[2];
  if (seg_finish<2>(acc, part, nchunks, g, s, S, tot) && threadIdx.x == 0) {
    S[s].rr = tot[0];
    S[s].bb = tot[1];
  }
}

// r32 = r / ||r|| (0 for systems not active), d = 0 (FP64 partial solution)
__global__ __launch_bounds__(256) void k_bto32(int nchunks, Seg g, const double* __restrict__ r,
                                               const double* __restrict__ scale,
                                               float* __restrict__ r32, double* __restrict__ d32) {
  SEG_PROLOGUE;
  const double inv = scale[s] > 0.0 ? 1.0 / scale[s] : 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += kBT) {
    r32[i] = (float)(r[i] * inv);
    d32[i] = 0.0;
  }
}

__global__ __launch_bounds__(256) void k_badd32(int nchunks, Seg g, double* __restrict__ x,
                                                const double* __restrict__ d,
                                                const double* __restrict__ scale) {
  SEG_PROLOGUE;
  const double sc = scale[s];
  if (sc == 0.0) return;
  for (int64_t i = lo + threadIdx.x; i < hi; i += kBT) x[i] += sc * (double)d[i];
}

__global__ void k_bset_active(BScal* S, int nsys, const int* active) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < nsys) S[s].active = active[s];
}

__global__ void k_bscal_reset(BScal* S, int nsys, const int* active) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nsys) return;
  S[s].it = 0;
  S[s].done = active[s] ? 0 : 1;
  S[s].active = active[s];
  S[s].breakdown = 0;
  S[s].counter = 0;
}

}  // namespace cpm

// ================================================================== host
struct cpm_batch {
  std::vector<cpm_band*> bands;
  int ninst = 0, nrhs = 1, dim = 3;
  std::unique_ptr<cpm_band> comp;
  std::vector<int64_t> D;                 // DOF offsets, [ninst + 1]
  int64_t total = 0;
  // segmented layout of the nrhs * ninst systems
  int nsys = 0, nchunks = 0;
  int* csys = nullptr;
  int64_t* clo = nullptr;
  int64_t* chi = nullptr;
  int* sfirst = nullptr;
  int* snch = nullptr;
  std::vector<int> h_csys;
  // per instance, the range of the composite's blocks and of its explicit FD
  // rows ([ninst + 1] each): the partials of a dot product fused into the
  // composite apply that belong to the instance
  std::vector<int> h_boff, h_loff;
  int* boff = nullptr;
  int* loff = nullptr;
  std::vector<double> m, n;
  cpm::DevAlloc da;                       // provider of the batch's device memory
  std::vector<std::pair<void*, size_t>> allocs;
  ~cpm_batch() {
    comp.reset();   // the composite band waits for the device if da is the caller's
    for (auto& pb : allocs) da.put(pb.first, pb.second);
  }
};

namespace cpm {
namespace {

using Clock = std::chrono::steady_clock;

template <class T>
T* dalloc(cpm_batch* B, size_t n) {
  const size_t bytes = (n ? n : 1) * sizeof(T);
  void* p = B->da.get(bytes);
  B->allocs.push_back({p, bytes});
  return static_cast<T*>(p);
}

void build_composite(cpm_batch* B, hipStream_t st) {
  const int ni = B->ninst;
  auto c = std::make_unique<cpm_band>();
  c->da = B->da;
  const cpm_band* b0 = B->bands[0];
  c->dim = b0->dim;
  c->N = b0->N;
  c->p = b0->p;
  c->composite = true;
  int64_t nb = 0, nt = 0, ntr = 0, ne = 0, nl = 0;
  B->D.assign(ni + 1, 0);
  for (int i = 0; i < ni; ++i) {
    const cpm_band* b = B->bands[i];
    if (b->dim != c->dim) CPM_FAIL(CPM_E_INVALID, "a batch needs bands of one dimension");
    if (b->p != c->p) CPM_FAIL(CPM_E_INVALID, "a batch needs bands of one interpolation degree");
    B->D[i + 1] = B->D[i] + b->n;
    nb += b->nb;
    nt += b->ntiles;
    ntr += b->n_tile_rows;
    ne += b->n_erows;
    nl += b->n_lrows;
  }
  B->total = B->D[ni];
  if (B->total * B->nrhs >= (1ll << 31)) CPM_FAIL(CPM_E_INVALID, "batch too large");
  const int d = c->dim, nm = d == 3 ? 64 : 16, nf = 2 * d;
  c->n = c->n_s = B->total;
  c->nb = (int)nb;
  c->ntiles = (int)nt;
  c->n_tile_rows = (int)ntr;
  c->n_erows = (int)ne;
  c->n_lrows = (int)nl;
  c->blk_face = c->alloc<QMeta>((size_t)nb * 8);
  c->tile_meta = c->alloc<QMeta>((size_t)nt * 8);
  c->tile_start = c->alloc<int>(nt + 1);
  c->perm = c->alloc<int>(ntr);
  c->frac64 = c->alloc<double>((size_t)d * ntr);
  c->frac32 = c->alloc<float>((size_t)d * ntr);
  c->lbase = c->alloc<unsigned>(ntr);
  c->erow_id = c->alloc<int>(ne);
  c->ecol = c->alloc<int>((size_t)ne * nm);
  c->ew = c->alloc<double>((size_t)ne * nm);
  c->ew32 = c->alloc<float>((size_t)ne * nm);
  c->lrow_id = c->alloc<int>(nl);
  c->lcol = c->alloc<int>((size_t)nl * nf);
  c->lrow_inst = c->alloc<int>(nl);
  c->erow_inst = c->alloc<int>(ne);
  c->tile_inst = c->alloc<int>(nt);
  c->inst_skip = c->alloc<int>((size_t)ni * B->nrhs);
  c->skip_stride = ni;
  CPM_HIP(hipMemsetAsync(c->inst_skip, 0, sizeof(int) * ni * B->nrhs, st));
  c->inst_coef = c->alloc<double>((size_t)2 * ni);
  int64_t ob = 0, ot = 0, otr = 0, oe = 0, ol = 0;
  B->h_boff.assign(ni + 1, 0);
  B->h_loff.assign(ni + 1, 0);
  auto g = [](int64_t n) { return dim3(grid_for(n, 256)); };
  for (int i = 0; i < ni; ++i) {
    const cpm_band* b = B->bands[i];
    const int add = (int)B->D[i];
    hipLaunchKernelGGL(k_cat_meta, g((int64_t)b->nb * 8), dim3(256), 0, st, b->blk_face,
                       c->blk_face + ob * 8, (int64_t)b->nb * 8, add, i);
    hipLaunchKernelGGL(k_cat_meta, g((int64_t)b->ntiles * 8), dim3(256), 0, st, b->tile_meta,
                       c->tile_meta + ot * 8, (int64_t)b->ntiles * 8, add, -1);
    hipLaunchKernelGGL(k_cat_int, g(b->ntiles), dim3(256), 0, st, b->tile_start,
                       c->tile_start + ot, (int64_t)b->ntiles, (int)otr);
    hipLaunchKernelGGL(k_cat_int, g(b->n_tile_rows), dim3(256), 0, st, b->perm, c->perm + otr,
                       (int64_t)b->n_tile_rows, add);
    for (int a = 0; a < d; ++a) {
      CPM_HIP(hipMemcpyAsync(c->frac64 + (int64_t)a * ntr + otr, b->frac64 + (int64_t)a * b->n_tile_rows,
                             sizeof(double) * b->n_tile_rows, hipMemcpyDeviceToDevice, st));
      CPM_HIP(hipMemcpyAsync(c->frac32 + (int64_t)a * ntr + otr, b->frac32 + (int64_t)a * b->n_tile_rows,
                             sizeof(float) * b->n_tile_rows, hipMemcpyDeviceToDevice, st));
    }
    CPM_HIP(hipMemcpyAsync(c->lbase + otr, b->lbase, sizeof(unsigned) * b->n_tile_rows,
                           hipMemcpyDeviceToDevice, st));
    hipLaunchKernelGGL(k_cat_int, g(b->n_erows), dim3(256), 0, st, b->erow_id, c->erow_id + oe,
                       (int64_t)b->n_erows, add);
    hipLaunchKernelGGL(k_cat_int, g((int64_t)b->n_erows * nm), dim3(256), 0, st, b->ecol,
                       c->ecol + oe * nm, (int64_t)b->n_erows * nm, add);
    CPM_HIP(hipMemcpyAsync(c->ew + oe * nm, b->ew, sizeof(double) * b->n_erows * nm,
                           hipMemcpyDeviceToDevice, st));
    CPM_HIP(hipMemcpyAsync(c->ew32 + oe * nm, b->ew32, sizeof(float) * b->n_erows * nm,
                           hipMemcpyDeviceToDevice, st));
    hipLaunchKernelGGL(k_cat_int, g(b->n_lrows), dim3(256), 0, st, b->lrow_id, c->lrow_id + ol,
                       (int64_t)b->n_lrows, add);
    hipLaunchKernelGGL(k_cat_int, g((int64_t)b->n_lrows * nf), dim3(256), 0, st, b->lcol,
                       c->lcol + ol * nf, (int64_t)b->n_lrows * nf, add);
    hipLaunchKernelGGL(k_fill_int, g(b->n_lrows), dim3(256), 0, st, c->lrow_inst + ol,
                       (int64_t)b->n_lrows, i);
    hipLaunchKernelGGL(k_fill_int, g(b->n_erows), dim3(256), 0, st, c->erow_inst + oe,
                       (int64_t)b->n_erows, i);
    hipLaunchKernelGGL(k_fill_int, g(b->ntiles), dim3(256), 0, st, c->tile_inst + ot,
                       (int64_t)b->ntiles, i);
    CPM_LAUNCH_CHECK();
    B->h_boff[i] = (int)ob;
    B->h_loff[i] = (int)ol;
    ob += b->nb;
    ot += b->ntiles;
    otr += b->n_tile_rows;
    oe += b->n_erows;
    ol += b->n_lrows;
  }
  const int ntr32 = (int)ntr;
  CPM_HIP(hipMemcpyAsync(c->tile_start + nt, &ntr32, sizeof(int), hipMemcpyHostToDevice, st));
  std::vector<double> coef(2 * ni);
  for (int i = 0; i < ni; ++i) {
    const double N2 = (double)B->bands[i]->N * (double)B->bands[i]->N;
    coef[2 * i] = B->m[i] + B->n[i] * (-2.0 * d * N2);
    coef[2 * i + 1] = B->n[i] * N2;
  }
  CPM_HIP(hipMemcpyAsync(c->inst_coef, coef.data(), sizeof(double) * 2 * ni,
                         hipMemcpyHostToDevice, st));
  B->h_boff[ni] = (int)ob;
  B->h_loff[ni] = (int)ol;
  B->boff = dalloc<int>(B, ni + 1);
  B->loff = dalloc<int>(B, ni + 1);
  CPM_HIP(hipMemcpyAsync(B->boff, B->h_boff.data(), sizeof(int) * (ni + 1),
                         hipMemcpyHostToDevice, st));
  CPM_HIP(hipMemcpyAsync(B->loff, B->h_loff.data(), sizeof(int) * (ni + 1),
                         hipMemcpyHostToDevice, st));
  CPM_HIP(hipStreamSynchronize(st));
  c->tune[0] = b0->tune[0];
  c->tune[1] = b0->tune[1];
  B->comp = std::move(c);

  // segmented layout: system s = r * ninst + i
  B->nsys = ni * B->nrhs;
  std::vector<int> csys, sfirst(B->nsys), snch(B->nsys);
  std::vector<int64_t> clo, chi;
  for (int r = 0; r < B->nrhs; ++r)
    for (int i = 0; i < ni; ++i) {
      const int s = r * ni + i;
      const int64_t base = (int64_t)r * B->total + B->D[i], len = B->D[i + 1] - B->D[i];
      sfirst[s] = (int)csys.size();
      for (int64_t o = 0; o < len; o += kChunk) {
        csys.push_back(s);
        clo.push_back(base + o);
        chi.push_back(base + std::min<int64_t>(len, o + kChunk));
      }
      snch[s] = (int)csys.size() - sfirst[s];
    }
  B->nchunks = (int)csys.size();
  B->csys = dalloc<int>(B, csys.size());
  B->clo = dalloc<int64_t>(B, clo.size());
  B->chi = dalloc<int64_t>(B, chi.size());
  B->sfirst = dalloc<int>(B, B->nsys);
  B->snch = dalloc<int>(B, B->nsys);
  CPM_HIP(hipMemcpy(B->csys, csys.data(), sizeof(int) * csys.size(), hipMemcpyHostToDevice));
  CPM_HIP(hipMemcpy(B->clo, clo.data(), sizeof(int64_t) * clo.size(), hipMemcpyHostToDevice));
  CPM_HIP(hipMemcpy(B->chi, chi.data(), sizeof(int64_t) * chi.size(), hipMemcpyHostToDevice));
  CPM_HIP(hipMemcpy(B->sfirst, sfirst.data(), sizeof(int) * B->nsys, hipMemcpyHostToDevice));
  CPM_HIP(hipMemcpy(B->snch, snch.data(), sizeof(int) * B->nsys, hipMemcpyHostToDevice));
  B->h_csys = csys;
}

// scratch slots of the composite band holding cpm_batch_autotune's vectors
constexpr int kAutotuneSlot = 90;

Seg seg_of(const cpm_batch* B) { return Seg{B->csys, B->clo, B->chi, B->sfirst, B->snch}; }

struct PinnedB {
  BScal* h = nullptr;
  explicit PinnedB(int n) { CPM_HIP(hipHostMalloc((void**)&h, sizeof(BScal) * n, hipHostMallocDefault)); }
  ~PinnedB() { if (h) (void)hipHostFree(h); }
};

// Segmented BiCGSTAB over every system of the batch (vectors [nrhs][total]);
// the iterate is of type TX (FP64 for the FP32 recurrence of mixed mode).
template <class T, class TX = T>
struct BBicg {
  cpm_batch* B;
  hipStream_t st;
  int64_t len;
  T *r, *rh, *p, *v, *s, *t;
  double* part;
  double* dpart;   // partials of the dot products fused into the applies
  int dnp = 0, lp0 = 0;
  BScal* S;
  int* act;
  PinnedB pin;
  std::vector<int> hact;
  hipGraphExec_t gexec = nullptr;
  int giters = 0;
  TX* gx = nullptr;

  BBicg(cpm_batch* b_, hipStream_t st_, int slot0)
      : B(b_), st(st_), len(b_->total * b_->nrhs), pin(b_->nsys), hact(b_->nsys, 1) {
    const cpm_band* c = B->comp.get();
    const size_t vb = sizeof(T) * (size_t)len;
    r = (T*)band_scratch(c, slot0, vb);
    rh = (T*)band_scratch(c, slot0 + 1, vb);
    p = (T*)band_scratch(c, slot0 + 2, vb);
    v = (T*)band_scratch(c, slot0 + 3, vb);
    s = (T*)band_scratch(c, slot0 + 4, vb);
    t = (T*)band_scratch(c, slot0 + 5, vb);
    part = (double*)band_scratch(c, slot0 + 6, sizeof(double) * 2 * B->nchunks);
    S = (BScal*)band_scratch(c, slot0 + 7, sizeof(BScal) * B->nsys);
    act = (int*)band_scratch(c, slot0 + 8, sizeof(int) * B->nsys);
    dnp = apply_dot_parts(c, false, sizeof(T) == 4);
    lp0 = dnp - 128 * (c->n_lrows ? grid_for(c->n_lrows, 128) : 0);
    dpart = (double*)band_scratch(c, slot0 + 9, sizeof(double) * 2 * (size_t)dnp * B->nrhs);
    CPM_HIP(hipMemsetAsync(S, 0, sizeof(BScal) * B->nsys, st));
    band_scratch(c, 0, apply_scratch_bytes(c, B->nrhs));
    set_active(hact);
  }
  ~BBicg() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
  }
  // out = A in; with dy, also the partials of (dy, out) and (out, out)
  void apply(const T* in, T* out, const T* dy = nullptr) {
    apply_impl<T>(B->comp.get(), 0.0, 0.0, B->nrhs, in, out, st, nullptr, 0.0, dy,
                  dy ? dpart : nullptr);
  }
  void set_active(const std::vector<int>& a) {
    hact = a;
    CPM_HIP(hipMemcpyAsync(act, hact.data(), sizeof(int) * B->nsys, hipMemcpyHostToDevice, st));
    CPM_HIP(hipStreamSynchronize(st));
  }
  void init(const T* rhs, const TX* x, bool x_zero, double tol) {
    hipLaunchKernelGGL(k_bscal_reset, dim3((B->nsys + 127) / 128), dim3(128), 0, st, S, B->nsys, act);
    if (!x_zero) {
      if constexpr (std::is_same<T, TX>::value) apply(x, v);
      else CPM_FAIL(CPM_E_INVALID, "internal: warm start of a mixed-type recurrence");
    }
    hipLaunchKernelGGL(k_binit<T>, dim3(B->nchunks), dim3(kBT), 0, st, B->nchunks, seg_of(B), rhs,
                       v, x_zero ? 0 : 1, r, rh, p, part, S, tol);
    CPM_LAUNCH_CHECK();
  }
  void iteration(TX* x) {
    const Seg g = seg_of(B);
    const int nc = B->nchunks;
    const int ns = B->nsys, ni = B->ninst;
    // the dot products (rh, v) and (s, t), (t, t) are fused into the applies
    apply(p, v, rh);
    hipLaunchKernelGGL(k_bdot_fin<0>, dim3(ns), dim3(kBT), 0, st, ni, dpart, dnp, lp0, B->boff,
                       B->loff, S);
    hipLaunchKernelGGL(k_bs<T>, dim3(nc), dim3(kBT), 0, st, nc, g, r, v, s, S);
    apply(s, t, s);
    hipLaunchKernelGGL(k_bdot_fin<1>, dim3(ns), dim3(kBT), 0, st, ni, dpart, dnp, lp0, B->boff,
                       B->loff, S);
    hipLaunchKernelGGL((k_bxr<T, TX>), dim3(nc), dim3(kBT), 0, st, nc, g, x, p, s, t, r, rh, part,
                       S);
    hipLaunchKernelGGL(k_bp<T>, dim3(nc), dim3(kBT), 0, st, nc, g, r, p, v, S);
    CPM_LAUNCH_CHECK();
  }
  void run(TX* x, int k, bool graph) {
    if (!graph) {
      for (int i = 0; i < k; ++i) iteration(x);
      return;
    }
    if (!gexec || giters != k || gx != x) {
      if (gexec) CPM_HIP(hipGraphExecDestroy(gexec));
      gexec = nullptr;
      hipGraph_t gr;
      CPM_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
      try {
        for (int i = 0; i < k; ++i) iteration(x);
      } catch (...) {
        // end the capture and drop what it recorded before passing the error on
        hipGraph_t part = nullptr;
        if (hipStreamEndCapture(st, &part) == hipSuccess && part) (void)hipGraphDestroy(part);
        throw;
      }
      CPM_HIP(hipStreamEndCapture(st, &gr));
      const hipError_t e = hipGraphInstantiate(&gexec, gr, nullptr, nullptr, 0);
      (void)hipGraphDestroy(gr);
      CPM_HIP(e);
      giters = k;
      gx = x;
    }
    CPM_HIP(hipGraphLaunch(gexec, st));
  }
  const BScal* read() {
    CPM_HIP(hipMemcpyAsync(pin.h, S, sizeof(BScal) * B->nsys, hipMemcpyDeviceToHost, st));
    CPM_HIP(hipStreamSynchronize(st));
    return pin.h;
  }
  // Returns the largest iteration count over the systems.
  int solve(const T* rhs, TX* x, bool x_zero, double tol, int maxit, int ce, bool graph) {
    init(rhs, x, x_zero, tol);
    const BScal* h = read();
    int it = 0;
    for (int restarts = 0;;) {
      bool all = true;
      std::vector<int> rs(B->nsys, 0);
      bool any_rs = false;
      for (int q = 0; q < B->nsys; ++q) {
        if (!h[q].done) all = false;
        rs[q] = hact[q] && h[q].done && h[q].breakdown && !(h[q].rr <= h[q].tol2);
        any_rs |= rs[q] != 0;
        it = std::max(it, h[q].it);
      }
      // restart the broken-down systems from their current iterate; the
      // others keep their recurrences (k_binit only touches active ones).
      // A mixed-type recurrence (an FP32 refinement step) ends instead: the
      // refinement loop restarts it from the FP64 residual.
      if constexpr (std::is_same<T, TX>::value) if (any_rs && restarts < 50) {
        ++restarts;
        clear_skip();   // the restart's apply must cover every instance
        const std::vector<int> keep = hact;
        set_active(rs);
        hipLaunchKernelGGL(k_bset_active, dim3((B->nsys + 127) / 128), dim3(128), 0, st, S,
                           B->nsys, act);
        apply(x, v);
        hipLaunchKernelGGL(k_binit<T>, dim3(B->nchunks), dim3(kBT), 0, st, B->nchunks, seg_of(B),
                           rhs, v, 1, r, rh, p, part, S, tol);
        set_active(keep);
        hipLaunchKernelGGL(k_bset_active, dim3((B->nsys + 127) / 128), dim3(128), 0, st, S,
                           B->nsys, act);
        CPM_LAUNCH_CHECK();
        h = read();
        continue;
      }
      if (all || it >= maxit) break;
      update_skip(h);
      run(x, std::min(ce, maxit - it), graph && std::min(ce, maxit - it) == ce);
      h = read();
    }
    clear_skip();
    return it;
  }
  // converged systems (instance, right-hand side) are skipped by the apply
  // kernels, which run one launch per right-hand side (system q = r * ninst
  // + i is flag q)
  void update_skip(const BScal* h) {
    std::vector<int> sk(B->nsys, 1);
    for (int q = 0; q < B->nsys; ++q)
      if (!h[q].done) sk[q] = 0;
    if (sk != hskip) {
      hskip = sk;
      CPM_HIP(hipMemcpyAsync(B->comp->inst_skip, hskip.data(), sizeof(int) * B->nsys,
                             hipMemcpyHostToDevice, st));
      CPM_HIP(hipStreamSynchronize(st));
    }
  }
  void clear_skip() {
    hskip.assign(B->nsys, 0);
    CPM_HIP(hipMemsetAsync(B->comp->inst_skip, 0, sizeof(int) * B->nsys, st));
    CPM_HIP(hipStreamSynchronize(st));
  }
  std::vector<int> hskip;
};

}  // namespace
}  // namespace cpm

using namespace cpm;

extern "C" cpm_status cpm_batch_create(cpm_band* const* bands, int nbands, const double* m,
                                       const double* n, int nrhs, const cpm_allocator* allocator,
                                       void* hip_stream, cpm_batch** out) {
  return guard([&] {
    if (!bands || nbands < 1 || !m || !n || nrhs < 1 || !out) CPM_FAIL(CPM_E_INVALID, "bad argument");
    if (allocator && (!allocator->alloc || !allocator->free))
      CPM_FAIL(CPM_E_INVALID, "an allocator needs both alloc and free");
    *out = nullptr;
    std::unique_ptr<cpm_batch> B(new cpm_batch());
    if (allocator) B->da.a = *allocator;
    B->da.st = (hipStream_t)hip_stream;
    for (int i = 0; i < nbands; ++i) {
      if (!bands[i]) CPM_FAIL(CPM_E_INVALID, "null band %d", i);
      B->bands.push_back(bands[i]);
      B->m.push_back(m[i]);
      B->n.push_back(n[i]);
    }
    B->ninst = nbands;
    B->nrhs = nrhs;
    build_composite(B.get(), (hipStream_t)hip_stream);
    *out = B.release();
  });
}

extern "C" void cpm_batch_free(cpm_batch* b) { delete b; }

extern "C" cpm_status cpm_batch_offsets(const cpm_batch* b, int64_t* offsets) {
  return guard([&] {
    if (!b || !offsets) CPM_FAIL(CPM_E_INVALID, "null argument");
    for (int i = 0; i <= b->ninst; ++i) offsets[i] = b->D[i];
  });
}

extern "C" cpm_status cpm_batch_apply(const cpm_batch* b, int dtype, const void* u, void* v,
                                      void* hip_stream) {
  return guard([&] {
    if (!b || !u || !v || u == v) CPM_FAIL(CPM_E_INVALID, "bad argument");
    hipStream_t st = (hipStream_t)hip_stream;
    if (dtype == CPM_F64)
      apply_impl<double>(b->comp.get(), 0.0, 0.0, b->nrhs, (const double*)u, (double*)v, st);
    else if (dtype == CPM_F32)
      apply_impl<float>(b->comp.get(), 0.0, 0.0, b->nrhs, (const float*)u, (float*)v, st);
    else
      CPM_FAIL(CPM_E_INVALID, "unknown dtype %d", dtype);
  });
}

extern "C" cpm_status cpm_batch_autotune(cpm_batch* b, int dtype, int reps, void* hip_stream,
                                         double* ms, int* best) {
  return guard([&] {
    if (!b) CPM_FAIL(CPM_E_INVALID, "null batch");
    if (dtype != CPM_F64 && dtype != CPM_F32) CPM_FAIL(CPM_E_INVALID, "unknown dtype %d", dtype);
    const size_t es = dtype == CPM_F64 ? 8 : 4;
    const size_t bytes = es * (size_t)b->total * b->nrhs;
    // the timing vectors are scratch of the composite band (kept for reuse)
    void* u = band_scratch(b->comp.get(), kAutotuneSlot, bytes);
    void* v = band_scratch(b->comp.get(), kAutotuneSlot + 1, bytes);
    CPM_HIP(hipMemsetAsync(u, 0, bytes, (hipStream_t)hip_stream));
    const cpm_status s = cpm_autotune(b->comp.get(), dtype, b->nrhs, u, v, reps, hip_stream, ms, best);
    if (s != CPM_OK) throw Error{s};
  });
}

// x (in: x0; out: solution) and rhs are [nrhs][total] double.  stats, when
// given, has nrhs * nbands entries (system s = r * nbands + i).
extern "C" cpm_status cpm_batch_solve(cpm_batch* b, const cpm_solve_opts* o, const double* rhs,
                                      double* x, cpm_solve_stats* stats, void* hip_stream) {
  cpm_status ret = CPM_OK;
  const cpm_status gs = guard([&] {
    if (!b || !o || !rhs || !x) CPM_FAIL(CPM_E_INVALID, "bad argument");
    if (o->gauge != 0.0) CPM_FAIL(CPM_E_INVALID, "the gauge is not supported in batches");
    const auto t0 = Clock::now();
    CPM_HIP(hipStreamSynchronize((hipStream_t)hip_stream));
    hipStream_t st = nullptr;
    CPM_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    struct SG {
      hipStream_t s;
      ~SG() { (void)hipStreamSynchronize(s); (void)hipStreamDestroy(s); }
    } sg{st};
    const cpm_band* c = b->comp.get();
    const int ns = b->nsys;
    const int64_t len = b->total * b->nrhs;
    const int maxit = o->maxit > 0 ? o->maxit : 20000;
    const int ce = o->check_every > 0 ? o->check_every : 16;
    const double tol = o->tol > 0 ? o->tol : 1e-8;
    const bool graph = o->use_graph != 0;
    double* r64 = (double*)band_scratch(c, 40, sizeof(double) * len);
    double* v64 = (double*)band_scratch(c, 41, sizeof(double) * len);
    double* part = (double*)band_scratch(c, 42, sizeof(double) * 2 * b->nchunks);
    BScal* S = (BScal*)band_scratch(c, 43, sizeof(BScal) * ns);
    double* scale = (double*)band_scratch(c, 44, sizeof(double) * ns);
    CPM_HIP(hipMemsetAsync(S, 0, sizeof(BScal) * ns, st));
    PinnedB pin(ns);
    std::vector<double> relres(ns, 0.0);
    std::vector<int> conv(ns, 0), iters(ns, 0), outer(ns, 0), fb(ns, 0);
    auto residual = [&]() {
      apply_impl<double>(c, 0.0, 0.0, b->nrhs, x, v64, st);
      hipLaunchKernelGGL(k_bres64, dim3(b->nchunks), dim3(kBT), 0, st, b->nchunks, seg_of(b), rhs,
                         v64, r64, part, S);
      CPM_LAUNCH_CHECK();
      CPM_HIP(hipMemcpyAsync(pin.h, S, sizeof(BScal) * ns, hipMemcpyDeviceToHost, st));
      CPM_HIP(hipStreamSynchronize(st));
      for (int q = 0; q < ns; ++q) {
        relres[q] = pin.h[q].bb > 0 ? std::sqrt(pin.h[q].rr / pin.h[q].bb) : 0.0;
        conv[q] = relres[q] <= tol;
      }
    };
    auto plain64 = [&](std::vector<int> active) {
      BBicg<double> k(b, st, 60);
      for (int rep = 0; rep < 20; ++rep) {
        bool any = false;
        for (int q = 0; q < ns; ++q) any |= active[q] != 0;
        if (!any) break;
        k.set_active(active);
        const int it = k.solve(rhs, x, false, tol, maxit, ce, graph);
        const BScal* h = k.read();
        for (int q = 0; q < ns; ++q)
          if (active[q]) iters[q] += h[q].it;
        (void)it;
        residual();
        for (int q = 0; q < ns; ++q) {
          if (active[q]) ++outer[q];
          active[q] = active[q] && !conv[q];
        }
      }
    };
    if (o->mode == CPM_SOLVE_F64) {
      plain64(std::vector<int>(ns, 1));
    } else {
      // FP32 refinement steps: each system's step solves A d = r / ||r|| with
      // an FP32 recurrence (the FP32 apply computes in FP64) to the relative
      // tolerance itol or kStepIters iterations, then x += ||r|| d in FP64.  A
      // system whose FP64 residual did not halve over a step finishes in FP64.
      const double itol = o->inner_tol > 0 ? o->inner_tol : 1e-2;
      constexpr int kStepIters = 1000;
      BBicg<float, double> k(b, st, 50);
      float* r32 = (float*)band_scratch(c, 45, sizeof(float) * len);
      double* d64 = (double*)band_scratch(c, 46, sizeof(double) * len);
      std::vector<double> h_scale(ns), prev(ns, HUGE_VAL);
      std::vector<int> active(ns, 1), failed(ns, 0);
      for (int step = 0; step < 100; ++step) {
        residual();
        bool any = false;
        for (int q = 0; q < ns; ++q) {
          if (active[q] && !conv[q] && !(relres[q] < 0.5 * prev[q])) failed[q] = 1;
          active[q] = active[q] && !conv[q] && !failed[q];
          prev[q] = relres[q];
          h_scale[q] = active[q] ? std::sqrt(pin.h[q].rr) : 0.0;
          any |= active[q] != 0;
        }
        if (!any) break;
        CPM_HIP(hipMemcpyAsync(scale, h_scale.data(), sizeof(double) * ns, hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(k_bto32, dim3(b->nchunks), dim3(kBT), 0, st, b->nchunks, seg_of(b), r64,
                           scale, r32, d64);
        CPM_LAUNCH_CHECK();
        k.set_active(active);
        k.solve(r32, d64, true, itol, kStepIters, ce, graph);
        const BScal* h = k.read();
        for (int q = 0; q < ns; ++q) {
          if (!active[q]) continue;
          iters[q] += h[q].it;
          ++outer[q];
          if (!(h[q].rr <= h[q].bb)) h_scale[q] = 0.0;   // diverged: drop the update
        }
        CPM_HIP(hipMemcpyAsync(scale, h_scale.data(), sizeof(double) * ns, hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(k_badd32, dim3(b->nchunks), dim3(kBT), 0, st, b->nchunks, seg_of(b), x,
                           d64, scale);
        CPM_LAUNCH_CHECK();
      }
      std::vector<int> rest(ns, 0);
      bool anyf = false;
      for (int q = 0; q < ns; ++q) {
        rest[q] = failed[q] && !conv[q];
        fb[q] = rest[q];
        anyf |= rest[q] != 0;
      }
      if (anyf) plain64(rest);
    }
    CPM_HIP(hipStreamSynchronize(st));
    const double ms = std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
    bool all = true;
    double worst = 0.0;
    for (int q = 0; q < ns; ++q) {
      all = all && conv[q];
      worst = std::max(worst, relres[q]);
      if (stats) {
        stats[q].converged = conv[q];
        stats[q].outer_iters = outer[q];
        stats[q].krylov_iters = iters[q];
        stats[q].restarts = 0;
        stats[q].fallback_f64 = fb[q];
        stats[q].relres = relres[q];
        stats[q].time_ms = ms;
      }
    }
    if (!all) {
      set_error("batched solve: some systems did not reach tol %.3g (worst %.3g)", tol, worst);
      ret = CPM_E_NOCONV;
    }
  });
  return gs != CPM_OK ? gs : ret;
}
