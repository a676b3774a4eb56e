// Error reporting, band lifetime and queries, workspace, device-wide scan.
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "cpm_internal.hpp"

namespace cpm {

namespace {
thread_local char g_err[1024] = "";
}

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

void* DevAlloc::get(size_t bytes) const {
  if (bytes == 0) bytes = 16;
  if (!custom()) {
    void* p = nullptr;
    CPM_HIP(hipMalloc(&p, bytes));
    return p;
  }
  void* p = a.alloc(bytes, (void*)st, a.ctx);
  if (!p) CPM_FAIL(CPM_E_OOM, "the caller's allocator returned NULL for %zu bytes", bytes);
  CPM_HIP(hipStreamSynchronize(st));
  return p;
}

void DevAlloc::put(void* p, size_t bytes) const noexcept {
  if (!p) return;
  if (!custom()) {
    (void)hipFree(p);
    return;
  }
  if (a.free) a.free(p, bytes ? bytes : 16, (void*)st, a.ctx);
}

void* Workspace::get(int i, size_t bytes) {
  if ((int)slots.size() <= i) slots.resize(i + 1, {nullptr, 0});
  auto& s = slots[i];
  if (s.second < bytes) {
    if (s.first) {
      // kernels of earlier calls may still read the old block (hipFree
      // waits for them by itself; a caller's allocator may not)
      if (da->custom()) CPM_HIP(hipDeviceSynchronize());
      da->put(s.first, s.second);
      total -= s.second;
    }
    s.first = nullptr;
    s.second = 0;
    s.first = da->get(bytes);
    s.second = bytes;
    total += bytes;
  }
  return s.first;
}

Workspace::~Workspace() {
  for (auto& s : slots) da->put(s.first, s.second);
}

void* band_scratch(const cpm_band* b, int slot, size_t bytes) {
  cpm_band* mb = const_cast<cpm_band*>(b);
  if (!mb->ws) {
    mb->ws = new Workspace();
    mb->ws->da = &mb->da;
  }
  return mb->ws->get(slot, bytes ? bytes : 16);
}

size_t band_scratch_bytes(const cpm_band* b) { return b->ws ? b->ws->total : 0; }

// ------------------------------------------------------------------- scan
// Exclusive prefix sum of int32 with an int64 total.  Each workgroup of 256
// threads scans 2048 items (8 per thread); workgroup totals are scanned
// recursively and added back.
constexpr int kScanItems = 8, kScanThreads = 256, kScanTile = kScanItems * kScanThreads;

__global__ __launch_bounds__(256) void k_scan_tile(const int* in, int* out, long long* sums,
                                                   int64_t n) {
  __shared__ long long s[kScanThreads];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  long long v[kScanItems];
  long long acc = 0;
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + k;
    v[k] = i < n ? in[i] : 0;
    acc += v[k];
  }
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 1; off < kScanThreads; off <<= 1) {
    long long t = threadIdx.x >= off ? s[threadIdx.x - off] : 0;
    __syncthreads();
    s[threadIdx.x] += t;
    __syncthreads();
  }
  long long run = s[threadIdx.x] - acc;   // exclusive prefix of this thread
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + k;
    if (i < n) out[i] = (int)run;
    run += v[k];
  }
  if (threadIdx.x == kScanThreads - 1) sums[blockIdx.x] = s[threadIdx.x];
}

__global__ __launch_bounds__(256) void k_scan_tile64(const long long* in, long long* out,
                                                     long long* sums, int64_t n) {
  __shared__ long long s[kScanThreads];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  long long v[kScanItems];
  long long acc = 0;
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + k;
    v[k] = i < n ? in[i] : 0;
    acc += v[k];
  }
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 1; off < kScanThreads; off <<= 1) {
    long long t = threadIdx.x >= off ? s[threadIdx.x - off] : 0;
    __syncthreads();
    s[threadIdx.x] += t;
    __syncthreads();
  }
  long long run = s[threadIdx.x] - acc;
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + k;
    if (i < n) out[i] = run;
    run += v[k];
  }
  if (threadIdx.x == kScanThreads - 1) sums[blockIdx.x] = s[threadIdx.x];
}

template <class T>
__global__ void k_scan_add(T* out, const long long* offs, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (T)((long long)out[i] + offs[i / kScanTile]);
}

namespace {
// scans 64-bit tile sums in place into exclusive offsets; returns the total
long long scan64_inplace(long long* a, int64_t n, hipStream_t st, const DevAlloc& da) {
  const int64_t nt = (n + kScanTile - 1) / kScanTile;
  const size_t sb = (nt + 1) * sizeof(long long);
  long long* sums = static_cast<long long*>(da.get(sb));
  long long total = 0;
  try {
    hipLaunchKernelGGL(k_scan_tile64, dim3(nt), dim3(kScanThreads), 0, st, a, a, sums, n);
    CPM_LAUNCH_CHECK();
    if (nt > 1) {
      total = scan64_inplace(sums, nt, st, da);
      hipLaunchKernelGGL(k_scan_add<long long>, dim3(grid_for(n, 256)), dim3(256), 0, st, a, sums, n);
      CPM_LAUNCH_CHECK();
    } else {
      CPM_HIP(hipMemcpyAsync(&total, sums, sizeof(long long), hipMemcpyDeviceToHost, st));
      CPM_HIP(hipStreamSynchronize(st));
    }
  } catch (...) {
    (void)hipStreamSynchronize(st);
    da.put(sums, sb);
    throw;
  }
  CPM_HIP(hipStreamSynchronize(st));
  da.put(sums, sb);
  return total;
}
}  // namespace

int64_t scan_exclusive_i32(const int* in, int* out, int64_t n, hipStream_t st,
                           const DevAlloc& da) {
  if (n <= 0) return 0;
  const int64_t nt = (n + kScanTile - 1) / kScanTile;
  const size_t sb = (nt + 1) * sizeof(long long);
  long long* sums = static_cast<long long*>(da.get(sb));
  long long total = 0;
  try {
    hipLaunchKernelGGL(k_scan_tile, dim3(nt), dim3(kScanThreads), 0, st, in, out, sums, n);
    CPM_LAUNCH_CHECK();
    if (nt > 1) {
      total = scan64_inplace(sums, nt, st, da);
      hipLaunchKernelGGL(k_scan_add<int>, dim3(grid_for(n, 256)), dim3(256), 0, st, out, sums, n);
      CPM_LAUNCH_CHECK();
    } else {
      CPM_HIP(hipMemcpyAsync(&total, sums, sizeof(long long), hipMemcpyDeviceToHost, st));
    }
    CPM_HIP(hipStreamSynchronize(st));
  } catch (...) {
    (void)hipStreamSynchronize(st);
    da.put(sums, sb);
    throw;
  }
  da.put(sums, sb);
  if (total >= (1ll << 31)) {
    set_error("scan total %lld exceeds the 32-bit index range", total);
    throw Error{CPM_E_INVALID};
  }
  return total;
}

}  // namespace cpm

cpm_band::~cpm_band() {
  // kernels on any stream may still read the band (hipFree would wait for
  // them by itself; a caller's allocator may hand the blocks out at once)
  if (da.custom()) (void)hipDeviceSynchronize();
  delete ws;
  for (auto& pb : allocs) da.put(pb.first, pb.second);
}

using namespace cpm;

extern "C" const char* cpm_last_error(void) { return g_err; }

extern "C" void cpm_band_free(cpm_band* band) { delete band; }

extern "C" cpm_status cpm_band_query(const cpm_band* b, cpm_band_info* out) {
  return guard([&] {
    if (!b || !out) CPM_FAIL(CPM_E_INVALID, "null argument");
    std::memset(out, 0, sizeof(*out));
    out->dim = b->dim;
    out->N = b->N;
    out->n_ibc = b->n_ibc;
    out->order = b->order;
    out->n_s = b->n_s;
    out->n_c = b->n_c;
    out->n = b->n;
    out->n_blocks = b->nb;
    out->n_tiles = b->ntiles;
    out->n_erows = b->n_erows;
    out->n_lrows = b->n_lrows;
    out->on_c_nodes = b->on_c_nodes;
    out->no_bc_dof_swaps = b->no_bc_dof_swaps;
    out->h = b->h;
    out->r_band = b->r;
    out->tau = b->tau;
    out->device_bytes = b->bytes;
    out->scratch_bytes = band_scratch_bytes(b);
  });
}
