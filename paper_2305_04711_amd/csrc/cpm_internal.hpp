// Internal declarations of libcpm (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/cpm.h"

namespace cpm {

// ------------------------------------------------------------------ errors
void set_error(const char* fmt, ...);

struct Error {
  cpm_status code;
};

#define CPM_HIP(call)                                                        \
  do {                                                                       \
    hipError_t e_ = (call);                                                  \
    if (e_ != hipSuccess) {                                                  \
      ::cpm::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), \
                       __FILE__, __LINE__);                                  \
      throw ::cpm::Error{e_ == hipErrorOutOfMemory ? CPM_E_OOM : CPM_E_HIP}; \
    }                                                                        \
  } while (0)

#define CPM_FAIL(code, ...)          \
  do {                               \
    ::cpm::set_error(__VA_ARGS__);   \
    throw ::cpm::Error{code};        \
  } while (0)

#define CPM_LAUNCH_CHECK() CPM_HIP(hipGetLastError())

// Runs f and converts exceptions into a status (no exception crosses the ABI).
template <class F>
cpm_status guard(F&& f) {
  try {
    f();
    return CPM_OK;
  } catch (const Error& e) {
    return e.code;
  } catch (const std::exception& e) {
    set_error("internal error: %s", e.what());
    return CPM_E_INVALID;
  } catch (...) {
    set_error("internal error");
    return CPM_E_INVALID;
  }
}

// --------------------------------------------------------------- geometry
// Block layout: 3-D blocks are 4x4x4 nodes, 2-D blocks 8x8 nodes; both hold
// 64 nodes, one wavefront, one 64-bit occupancy mask.  Slot s of a block:
// 3-D s = lx + 4 ly + 16 lz, 2-D s = lx + 8 ly.
template <int DIM> struct Geo;
template <> struct Geo<3> {
  static constexpr int BX = 4, SH = 2, NNBR = 27;
  __host__ __device__ static int slot(int lx, int ly, int lz) { return lx + 4 * ly + 16 * lz; }
  __host__ __device__ static int lx(int s) { return s & 3; }
  __host__ __device__ static int ly(int s) { return (s >> 2) & 3; }
  __host__ __device__ static int lz(int s) { return s >> 4; }
  __host__ __device__ static int code(int dx, int dy, int dz) { return (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1); }
};
template <> struct Geo<2> {
  static constexpr int BX = 8, SH = 3, NNBR = 9;
  __host__ __device__ static int slot(int lx, int ly, int) { return lx + 8 * ly; }
  __host__ __device__ static int lx(int s) { return s & 7; }
  __host__ __device__ static int ly(int s) { return s >> 3; }
  __host__ __device__ static int lz(int) { return 0; }
  __host__ __device__ static int code(int dx, int dy, int) { return (dy + 1) * 3 + (dx + 1); }
};

struct Workspace;

// Device memory of a band or batch: through the caller's cpm_allocator (with
// the stream given at creation), or hipMalloc / hipFree when none was given.
// get() throws CPM_E_OOM when the allocator fails; after a caller's
// allocation it synchronises that stream, so that no work the allocator's
// stream still had queued on the block overlaps the library's use of it on
// other streams.
struct DevAlloc {
  cpm_allocator a{};
  hipStream_t st = nullptr;
  bool custom() const { return a.alloc != nullptr; }
  void* get(size_t bytes) const;
  void put(void* p, size_t bytes) const noexcept;
};

// Occupancy mask and first DOF of one block (mask 0 when the block is absent).
struct QMeta {
  unsigned long long mask;
  int off;
  int pad;
};

// Launch variants of the apply kernels (chosen by the autotuner).
struct Tune {
  int pad = 1;     // LDS x-line stride of the staged cube: 0 -> E + 1, 1 -> E + 4
  int xcd = 1;     // map consecutive tiles / blocks to one XCD
  int ps = 0;      // tile gather as persistent wavefronts (implies xcd): 1
                   // prefetches the next tile's metadata, 2 also its staging
  int lap = 0;     // Laplacian pass: 0 gathers every neighbour, 1 exchanges
                   // in-block neighbours between lanes, 2 does so in
                   // persistent wavefronts that request the next block early,
                   // 3 keeps the metadata in scalar registers and exchanges
                   // with row moves and lane permutes (k_lap_w)
  int tuned = 0;
};
// variant k: pad = k & 1, order mode = (k >> 1) & 3 (0 block order, 1
// XCD-aware, 2 persistent XCD-aware gather, 3 persistent and pipelined),
// lap = k >> 3
constexpr int kTuneVariants = 32;
inline Tune tune_variant(int k) {
  Tune t;
  t.pad = k & 1;
  const int mode = (k >> 1) & 3;
  t.xcd = mode != 0;
  t.ps = mode >= 2 ? mode - 1 : 0;
  t.lap = k >> 3;
  t.tuned = 1;
  return t;
}
// Persistent tile gather: wavefronts per XCD (8 per SIMD at most are resident)
constexpr int kPersistWavesPerXcd = 4096;

}  // namespace cpm

// The band: everything a call needs, all arrays on the device.
struct cpm_band {
  int dim = 0, N = 0, order = 2, n_ibc = 0, p = 3;
  int band_kind = CPM_BAND_TUBE;
  cpm_surface surf{};
  std::vector<cpm_ibc> ibcs;
  double h = 0, r = 0, tau = 0, check_factor = 2;
  int64_t n_s = 0, n_c = 0, n = 0;
  int device = 0;

  // occupied blocks (block order = Morton order of the block coordinates)
  int nb = 0;
  int4* blk_coord = nullptr;          // [nb] block coordinates
  unsigned long long* blk_mask = nullptr;  // [nb] occupied slots
  int* blk_off = nullptr;             // [nb + 1] first PDE DOF of the block
  int* blk_nbr = nullptr;             // [nb][NNBR] neighbour block ids or -1
  unsigned long long* lrow_mask = nullptr; // [nb] slots whose L row is explicit
  // [nb][8] per-block Laplacian metadata: entry 0 the block itself, 1..2d its
  // face neighbours (-x,+x,-y,+y,-z,+z), 7 the explicit-row mask in .mask
  cpm::QMeta* blk_face = nullptr;

  // hash table block key -> block id (open addressing)
  unsigned long long* hkeys = nullptr;
  int* hvals = nullptr;
  unsigned int hcap = 0;

  // PDE rows
  double* cp = nullptr;               // [dim][n_s] stored cp_S (SoA)

  // gather tiles: PDE rows without swapped interpolation members, grouped by
  // the block that holds their stencil base
  int ntiles = 0, n_tile_rows = 0;
  int* tile_blk = nullptr;            // [ntiles]
  cpm::QMeta* tile_meta = nullptr;    // [ntiles][8] the 2^d staged blocks
  int* tile_start = nullptr;          // [ntiles + 1]
  int* perm = nullptr;                // [n_tile_rows] row DOF
  double* frac64 = nullptr;           // [dim][n_tile_rows] FP64 fractions
  float* frac32 = nullptr;            // [dim][n_tile_rows] FP32 fractions
  unsigned int* lbase = nullptr;      // [n_tile_rows] packed local base
  // tiles grouped by the parity class of their block (k_tile_colour): class
  // k is tile_col[col_start[k] .. col_start[k + 1]), each entry {tile, first
  // row, end row, 0} (the tile's range in the tile-row arrays)
  int4* tile_col = nullptr;           // [ntiles]
  int col_start[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};

  // rows with explicit interpolation stencils (swapped PDE rows, BC rows)
  int n_erows = 0;
  int* erow_id = nullptr;             // [n_erows]
  int* ecol = nullptr;                // [n_erows][4^dim]
  double* ew = nullptr;               // [n_erows][4^dim]
  float* ew32 = nullptr;              // [n_erows][4^dim]
  int* ebase = nullptr;               // [n_erows][dim]

  // rows with explicit FD stencils (swapped PDE rows, BC rows)
  int n_lrows = 0;
  int* lrow_id = nullptr;             // [n_lrows]
  int* lcol = nullptr;                // [n_lrows][2 dim] after swaps, -1 none
  int* lcol0 = nullptr;               // [n_lrows][2 dim] before swaps (PDE rows)

  // pull lists of the transposed explicit rows (single bands; a batch's
  // composite has none: batches apply only the forward operator): target DOFs, segment
  // starts and sources in ascending order per target.  E: per entry the DOF
  // of its row and its weight (et_src, et_w, et_w32; sources i * 4^d + o,
  // entry o of explicit E row i, in ascending order).  L: source 2 i + s,
  // explicit FD row i, s = 1 for the subtracted unswapped column of a
  // swapped PDE entry.
  int n_et = 0, n_lt = 0, n_et_entries = 0;
  int *et_tgt = nullptr, *et_start = nullptr, *et_src = nullptr;
  double* et_w = nullptr;
  float* et_w32 = nullptr;
  int *lt_tgt = nullptr, *lt_start = nullptr, *lt_src = nullptr;

  // BC DOFs
  int* bc_node = nullptr;             // [n_c]
  double* bc_cpc = nullptr;           // [n_c][dim]
  int* bc_side = nullptr;             // [n_c]
  int* bc_curve = nullptr;            // [n_c]
  double* bc_ecoef = nullptr;         // [n_c] multiplier of g in the row constant

  // composite of several bands (batched solves): per-instance FD
  // coefficients (cd, co) of A, instance of each explicit FD row
  double* inst_coef = nullptr;
  int* lrow_inst = nullptr;
  int* erow_inst = nullptr;           // instance of each explicit E row
  int* tile_inst = nullptr;           // instance of each tile
  int* inst_skip = nullptr;           // [nrhs][instances] 1: skip (that system is done)
  int skip_stride = 0;                // instances (row length of inst_skip)
  bool composite = false;

  int64_t on_c_nodes = 0, no_bc_dof_swaps = 0;
  size_t bytes = 0;
  cpm::DevAlloc da;                   // provider of every device allocation
  std::vector<std::pair<void*, size_t>> allocs;
  cpm::Workspace* ws = nullptr;
  cpm::Tune tune[2];                  // per dtype (0 = FP64, 1 = FP32)

  template <class T>
  T* alloc(size_t count) {
    size_t b = count * sizeof(T);
    if (b == 0) b = 16;
    void* p = da.get(b);
    allocs.push_back({p, b});
    bytes += b;
    return static_cast<T*>(p);
  }
  ~cpm_band();
};

namespace cpm {

// Scratch vectors owned by a band, grown on demand through the band's
// allocator (calls on one band from several threads at once race on them).
// A slot that grows is released after the device has finished its work.
struct Workspace {
  const DevAlloc* da = nullptr;
  size_t total = 0;
  std::vector<std::pair<void*, size_t>> slots;
  void* get(int i, size_t bytes);
  ~Workspace();
};
void* band_scratch(const cpm_band* b, int slot, size_t bytes);
size_t band_scratch_bytes(const cpm_band* b);

// Device-wide exclusive scan; returns the total (synchronises the stream).
// Its temporaries come from da.
int64_t scan_exclusive_i32(const int* in, int* out, int64_t n, hipStream_t s, const DevAlloc& da);

// apply entry points used by the solvers (nrhs = 1, optional gauge).  With
// dy set, the kernel that writes v also writes the partials of (dy, v) and
// (v, v) to dpart[0 .. np) and dpart[np .. 2 np), np = apply_dot_parts.
template <class T>
void apply_impl(const cpm_band* b, double m, double n, int nrhs, const T* u,
                T* v, hipStream_t s, const double* gauge_sum = nullptr,
                double gamma = 0.0, const T* dy = nullptr, double* dpart = nullptr);
template <class T>
void apply_transpose_impl(const cpm_band* b, double m, double n, int nrhs,
                          const T* w, T* z, hipStream_t s,
                          const double* gauge_sum = nullptr, double gamma = 0.0,
                          const T* dy = nullptr, double* dpart = nullptr);
int apply_dot_parts(const cpm_band* b, bool transpose, bool f32);
// bytes of the forward apply's scratch vector (the FP64 intermediate a = E u)
size_t apply_scratch_bytes(const cpm_band* b, int nrhs);
// out -= n (L - diag L) e(g): the Dirichlet part of a right-hand side
void add_dirichlet_term(const cpm_band* b, double n, const double* g, int nrhs, double* out,
                        hipStream_t st);

inline int grid_for(int64_t n, int threads, int cap = 1 << 20) {
  int64_t g = (n + threads - 1) / threads;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return static_cast<int>(g);
}

}  // namespace cpm
