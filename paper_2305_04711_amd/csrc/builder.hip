// Band builder: Omega(S) (eq. bandwidth; the set Algorithm 1 finds), interior
// boundary sets (Sec. 4.1, 4.6), side vectors (eq. cpdiff, Sec. 4.2), stencils
// with swaps (Sec. 4.3) and the gather tiles of the apply kernels.
//
// Storage is a sparse two-level grid (Sec. 5.1): occupied blocks of 64 nodes
// (4x4x4, or 8x8 in 2-D) found by scanning the bounding box one row of blocks
// per workgroup, a hash table from block coordinates to block ids, and a
// neighbour table per block.  Blocks are numbered in Morton (Z) order of
// their coordinates, so that blocks adjacent in any direction are close in
// the numbering (and in the order the apply kernels visit them); PDE DOFs are
// numbered block by block, slots in order inside a block.
//
// Compiled with -ffp-contract=off: every FP64 decision here must agree bit
// for bit with a plain IEEE evaluation of the same formulas.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>

#include <hipcub/hipcub.hpp>

#include "cpm_internal.hpp"
#include "geom.hpp"
#include "lagrange.hpp"

namespace cpm {

constexpr unsigned long long kEmpty = ~0ull;
constexpr int kMaxIBC = 8;

struct IBCList {
  cpm_ibc c[kMaxIBC];
  int n;
};

__host__ __device__ __forceinline__ unsigned long long block_key(int bx, int by, int bz) {
  return (unsigned long long)(unsigned)(bx + (1 << 20)) |
         ((unsigned long long)(unsigned)(by + (1 << 20)) << 21) |
         ((unsigned long long)(unsigned)(bz + (1 << 20)) << 42);
}

// Bits 0..20 of v moved to bits 0, 3, 6, ..., 60.
__host__ __device__ __forceinline__ unsigned long long spread3(unsigned v) {
  unsigned long long x = v & 0x1fffffu;
  x = (x | (x << 32)) & 0x001f00000000ffffULL;
  x = (x | (x << 16)) & 0x001f0000ff0000ffULL;
  x = (x | (x << 8)) & 0x100f00f00f00f00fULL;
  x = (x | (x << 4)) & 0x10c30c30c30c30c3ULL;
  x = (x | (x << 2)) & 0x1249249249249249ULL;
  return x;
}

// Morton key of a block: the offset coordinates' bits interleaved (x lowest).
__host__ __device__ __forceinline__ unsigned long long morton_key(int bx, int by, int bz) {
  return spread3((unsigned)(bx + (1 << 20))) | (spread3((unsigned)(by + (1 << 20))) << 1) |
         (spread3((unsigned)(bz + (1 << 20))) << 2);
}

__device__ __forceinline__ unsigned hash_key(unsigned long long k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdULL;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ULL;
  k ^= k >> 33;
  return (unsigned)k;
}

__device__ int hash_find(const unsigned long long* keys, const int* vals,
                         unsigned cap, unsigned long long key) {
  unsigned h = hash_key(key) & (cap - 1);
  for (unsigned probe = 0; probe < cap; ++probe) {
    const unsigned long long k = keys[h];
    if (k == key) return vals[h];
    if (k == kEmpty) return -1;
    h = (h + 1) & (cap - 1);
  }
  return -1;
}

// Read-only view of the block structure used by device helpers.
struct Blocks {
  const int4* coord;
  const unsigned long long* mask;
  const int* off;
  const int* nbr;
  const unsigned long long* hkeys;
  const int* hvals;
  unsigned hcap;
  int p;   // interpolation degree: 3 (cubic) or 2 (quadratic)
};

// DOF of the node at local coordinates (mx, my, mz) relative to block blk;
// each local coordinate may lie in [-BX, 2 BX).  -1 if not a band node.
template <int DIM>
__device__ __forceinline__ int node_dof(const Blocks& B, int blk, int mx, int my, int mz) {
  using G = Geo<DIM>;
  const int dx = mx >> G::SH, dy = my >> G::SH, dz = DIM == 3 ? (mz >> G::SH) : 0;
  int b = blk;
  if (dx | dy | dz) b = B.nbr[blk * G::NNBR + G::code(dx, dy, dz)];
  if (b < 0) return -1;
  const int s = G::slot(mx & (G::BX - 1), my & (G::BX - 1), DIM == 3 ? (mz & (G::BX - 1)) : 0);
  const unsigned long long m = B.mask[b];
  if (!((m >> s) & 1ull)) return -1;
  return B.off[b] + __popcll(m & ((1ull << s) - 1ull));
}

template <int DIM>
__device__ __forceinline__ int block_of(const Blocks& B, int kx, int ky, int kz) {
  using G = Geo<DIM>;
  return hash_find(B.hkeys, B.hvals, B.hcap,
                   block_key(kx >> G::SH, ky >> G::SH, DIM == 3 ? (kz >> G::SH) : 0));
}

// Stencil base and fraction of a query point (eq. interp-stencil): cubic,
// the nodes floor(y N) - 1 .. + 2 with t = y N - floor(y N); quadratic, the
// nearest nodes floor(y N + 1/2) - 1 .. + 1 with t = y N - floor(y N + 1/2).
// Either way the query lies at base + 1 + t.
template <int DIM>
__device__ __forceinline__ void stencil_base(const V3& y, int N, int p, int base[3], double t[3]) {
  const double dn = (double)N;
  const double s[3] = {y.x * dn, y.y * dn, y.z * dn};
  for (int a = 0; a < DIM; ++a) {
    const double F = p == 3 ? floor(s[a]) : floor(s[a] + 0.5);
    base[a] = (int)F - 1;
    t[a] = s[a] - F;
  }
  if (DIM == 2) {
    base[2] = 0;
    t[2] = 0.0;
  }
}

// ------------------------------------------------------------------ pass 1
struct Box {
  int blo[3];
  int nb[3];
};

// One workgroup per row of blocks (fixed by, bz); each wavefront classifies
// one block at a time, lane = slot.  WRITE = false counts occupied blocks per
// row; WRITE = true stores them in order at the row's offset.  With a filter
// (the stencil set, Sec. 5.1) a block keeps only the nodes of the filter's
// mask for the same block coordinates.
struct Filter {
  const unsigned long long* hkeys = nullptr;   // block hash of the filtering band
  const int* hvals = nullptr;
  unsigned hcap = 0;
  const unsigned long long* keep = nullptr;    // [its blocks] nodes to keep; null: no filter
};

template <int DIM, bool WRITE>
__global__ __launch_bounds__(256) void k_classify(cpm_surface S, int N, double r,
                                                  double thr, Box box, int* row_count,
                                                  const int* row_off, int4* out_coord,
                                                  unsigned long long* out_mask, Filter F) {
  using G = Geo<DIM>;
  const int row = blockIdx.x;
  const int by = box.blo[1] + row % box.nb[1];
  const int bz = DIM == 3 ? box.blo[2] + row / box.nb[1] : 0;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __shared__ unsigned long long s_mask[4];
  __shared__ int s_count;
  if (threadIdx.x == 0) s_count = 0;
  __syncthreads();
  const int nchunks = (box.nb[0] + 3) / 4;
  const double hc = 0.5 * (double)(G::BX - 1);
  const double dn = (double)N;
  for (int ch = 0; ch < nchunks; ++ch) {
    const int bxi = ch * 4 + wave;
    unsigned long long m = 0;
    if (bxi < box.nb[0]) {
      const int bx = box.blo[0] + bxi;
      // wave-uniform pre-test on the block centre; the distance to S is
      // 1-Lipschitz, so a centre farther than r + half diagonal has no node
      // within r (NaN compares false and falls through to the full test)
      const V3 c{((double)(bx * G::BX) + hc) / dn, ((double)(by * G::BX) + hc) / dn,
                 DIM == 3 ? ((double)(bz * G::BX) + hc) / dn : 0.0};
      const double dc = dist<DIM>(c, cp_surface<DIM>(S, c));
      if (!(dc > thr)) {
        const int kx = bx * G::BX + G::lx(lane);
        const int ky = by * G::BX + G::ly(lane);
        const int kz = DIM == 3 ? bz * G::BX + G::lz(lane) : 0;
        const V3 p = node_pos(kx, ky, kz, N);
        const bool in = dist<DIM>(p, cp_surface<DIM>(S, p)) <= r;
        m = __ballot(in);
        if (F.keep && m) {
          const int id = hash_find(F.hkeys, F.hvals, F.hcap, block_key(bx, by, DIM == 3 ? bz : 0));
          m &= id >= 0 ? F.keep[id] : 0ull;
        }
      }
    }
    if (lane == 0) s_mask[wave] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int w = 0; w < 4; ++w) {
        if (s_mask[w]) {
          if (WRITE) {
            const int pos = row_off[row] + s_count;
            out_coord[pos] = make_int4(box.blo[0] + ch * 4 + w, by, bz, 0);
            out_mask[pos] = s_mask[w];
          }
          ++s_count;
        }
      }
    }
    __syncthreads();
  }
  if (!WRITE && threadIdx.x == 0) row_count[row] = s_count;
}

__global__ void k_morton(const int4* coord, int nb, unsigned long long* key, int* idx) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nb) return;
  const int4 c = coord[i];
  key[i] = morton_key(c.x, c.y, c.z);
  idx[i] = i;
}

__global__ void k_permute_blocks(const int* idx, int nb, const int4* coord_in,
                                 const unsigned long long* mask_in, int4* coord,
                                 unsigned long long* mask) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nb) return;
  const int j = idx[i];
  coord[i] = coord_in[j];
  mask[i] = mask_in[j];
}

__global__ void k_popcounts(const unsigned long long* mask, int nb, int* cnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nb) cnt[i] = __popcll(mask[i]);
}

__global__ void k_hash_insert(const int4* coord, int nb, unsigned long long* keys,
                              int* vals, unsigned cap) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nb) return;
  const int4 c = coord[i];
  const unsigned long long key = block_key(c.x, c.y, c.z);
  unsigned h = hash_key(key) & (cap - 1);
  for (unsigned probe = 0; probe < cap; ++probe) {
    const unsigned long long prev = atomicCAS(&keys[h], kEmpty, key);
    if (prev == kEmpty || prev == key) {
      vals[h] = i;
      return;
    }
    h = (h + 1) & (cap - 1);
  }
}

template <int DIM>
__global__ void k_neighbours(Blocks B, int nb, int* nbr) {
  using G = Geo<DIM>;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)nb * G::NNBR) return;
  const int i = (int)(t / G::NNBR), c = (int)(t % G::NNBR);
  const int dx = c % 3 - 1, dy = (c / 3) % 3 - 1, dz = DIM == 3 ? c / 9 - 1 : 0;
  const int4 bc = B.coord[i];
  nbr[t] = hash_find(B.hkeys, B.hvals, B.hcap, block_key(bc.x + dx, bc.y + dy, bc.z + dz));
}

// Thread mapping of the per-node kernels: 4 blocks per workgroup, lane = slot.
#define NODE_PROLOGUE(DIMV)                                                   \
  using G = Geo<DIMV>;                                                        \
  const int blk = blockIdx.x * 4 + (threadIdx.x >> 6);                        \
  const int slot = threadIdx.x & 63;                                          \
  if (blk >= nb) return;                                                      \
  const unsigned long long msk = B.mask[blk];                                 \
  if (!((msk >> slot) & 1ull)) return;                                        \
  const int dof = B.off[blk] + __popcll(msk & ((1ull << slot) - 1ull));       \
  const int4 bcrd = B.coord[blk];                                             \
  const int kx = bcrd.x * G::BX + G::lx(slot);                                \
  const int ky = bcrd.y * G::BX + G::ly(slot);                                \
  const int kz = DIMV == 3 ? bcrd.z * G::BX + G::lz(slot) : 0;                \
  (void)kx; (void)ky; (void)kz; (void)dof

template <int DIM>
__global__ __launch_bounds__(256) void k_rows(Blocks B, int nb, cpm_surface S, int N,
                                              int64_t n_s, double* cp) {
  NODE_PROLOGUE(DIM);
  const V3 p = node_pos(kx, ky, kz, N);
  const V3 c = cp_surface<DIM>(S, p);
  cp[dof] = c.x;
  cp[n_s + dof] = c.y;
  if (DIM == 3) cp[2 * n_s + dof] = c.z;
}

__device__ __forceinline__ V3 load_v(const double* a, int64_t n_s, int i, int dim) {
  return V3{a[i], a[n_s + i], dim == 3 ? a[2 * n_s + i] : 0.0};
}

// Interior-boundary classification of every PDE node.
template <int DIM>
__global__ __launch_bounds__(256) void k_ibc_rows(Blocks B, int nb, cpm_surface S, IBCList L,
                                                  int N, int64_t n_s, double r, double cf,
                                                  double tau, const double* cp, int* row_c,
                                                  int* omega, double* side_v, double* cpcs,
                                                  unsigned long long* counters) {
  NODE_PROLOGUE(DIM);
  const V3 p = node_pos(kx, ky, kz, N);
  const V3 q = load_v(cp, n_s, dof, DIM);
  int rc = -1, om = 0;
  for (int c = 0; c < L.n; ++c) {
    // past the end of an open curve: neither BC DOFs nor stencil changes
    if (curve_at_end(S, L.c[c], p)) continue;
    const V3 pc = cp_curve<DIM>(S, L.c[c], p);
    const double dC = dist<DIM>(p, pc);
    if (dC < cf * r) {
      if (rc >= 0) atomicOr(&counters[2], 1ull);     // overlapping check regions
      rc = c;
      om = dC <= r ? 1 : 0;
      V3 v{q.x - pc.x, q.y - pc.y, q.z - pc.z};
      const double nv = sqrt(dot3<DIM>(v, v));
      if (nv < tau) {
        const V3 o = orient_curve<DIM>(S, L.c[c], pc);
        v = V3{tau * o.x, tau * o.y, tau * o.z};
        atomicAdd(&counters[0], 1ull);
      }
      side_v[dof] = v.x;
      side_v[n_s + dof] = v.y;
      cpcs[dof] = pc.x;
      cpcs[n_s + dof] = pc.y;
      if (DIM == 3) {
        side_v[2 * n_s + dof] = v.z;
        cpcs[2 * n_s + dof] = pc.z;
      }
    }
  }
  row_c[dof] = rc;
  omega[dof] = om;
}

__global__ void k_flag_curve(const int* row_c, const int* omega, int64_t n_s, int c, int* flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_s) flag[i] = (row_c[i] == c && omega[i]) ? 1 : 0;
}

template <int DIM>
__global__ __launch_bounds__(256) void k_bc_assign(Blocks B, int nb, const int* flag,
                                                   const int* rank, int64_t n_s,
                                                   int64_t base_alpha, int c, cpm_surface S,
                                                   IBCList L, const double* side_v,
                                                   const double* cpcs, int* alpha_of,
                                                   int* bc_node, double* bc_cpc, int* bc_side,
                                                   int* bc_curve, int* bc_k) {
  NODE_PROLOGUE(DIM);
  if (!flag[dof]) return;
  const int64_t a = base_alpha + rank[dof];   // BC DOF index minus n_s
  alpha_of[dof] = (int)(n_s + a);
  bc_node[a] = dof;
  bc_k[a * 3 + 0] = kx;
  bc_k[a * 3 + 1] = ky;
  bc_k[a * 3 + 2] = kz;
  const V3 pc = load_v(cpcs, n_s, dof, DIM);
  const V3 v = load_v(side_v, n_s, dof, DIM);
  bc_cpc[a * DIM + 0] = pc.x;
  bc_cpc[a * DIM + 1] = pc.y;
  if (DIM == 3) bc_cpc[a * DIM + 2] = pc.z;
  const V3 o = orient_curve<DIM>(S, L.c[c], pc);
  bc_side[a] = dot3<DIM>(v, o) < 0.0 ? -1 : 1;
  bc_curve[a] = c;
}

// Interpolation members of a PDE row: hole count, swap flag (eq.
// stencil-crossing-test), and the gather-tile count of rows without swaps.
template <int DIM>
__global__ __launch_bounds__(256) void k_stencil_scan(Blocks B, int nb, int N, int64_t n_s,
                                                      const double* cp, const int* row_c,
                                                      const int* alpha_of, const double* side_v,
                                                      int* eflag, int* tile_blk_of,
                                                      int* tile_cnt,
                                                      unsigned long long* counters) {
  NODE_PROLOGUE(DIM);
  const V3 y = load_v(cp, n_s, dof, DIM);
  int base[3];
  double t[3];
  stencil_base<DIM>(y, N, B.p, base, t);
  const int bb = block_of<DIM>(B, base[0], base[1], base[2]);
  const int lx = base[0] & (G::BX - 1), ly = base[1] & (G::BX - 1),
            lz = DIM == 3 ? (base[2] & (G::BX - 1)) : 0;
  const int rc = row_c ? row_c[dof] : -1;
  V3 vi{0, 0, 0};
  if (rc >= 0) vi = load_v(side_v, n_s, dof, DIM);
  int holes = 0, swaps = 0, nobc = 0;
  const int np = B.p + 1, nmp = DIM == 3 ? np * np * np : np * np;
  for (int o = 0; o < nmp; ++o) {
    const int a = o % np, b = (o / np) % np, c = o / (np * np);
    const int j = bb < 0 ? -1 : node_dof<DIM>(B, bb, lx + a, ly + b, lz + c);
    if (j < 0) {
      ++holes;
      continue;
    }
    if (rc >= 0 && row_c[j] == rc) {
      const V3 vj = load_v(side_v, n_s, j, DIM);
      if (dot3<DIM>(vi, vj) < 0.0) {
        if (alpha_of[j] >= 0) ++swaps;
        else ++nobc;
      }
    }
  }
  if (holes) atomicAdd(&counters[3], (unsigned long long)holes);
  if (nobc) atomicAdd(&counters[1], (unsigned long long)nobc);
  eflag[dof] = swaps ? 1 : 0;
  tile_blk_of[dof] = bb;
  if (!swaps && bb >= 0 && !holes) atomicAdd(&tile_cnt[bb], 1);
}

// Tile rows are ordered by their local stencil base inside the tile: rows
// along one surface normal share cp_S, hence the base, and neighbouring lanes
// then read identical LDS addresses (served as broadcasts).
template <int DIM>
__device__ __forceinline__ int local_base_code(const int base[3]) {
  using G = Geo<DIM>;
  const int lx = base[0] & (G::BX - 1), ly = base[1] & (G::BX - 1);
  return DIM == 3 ? lx + 4 * ly + 16 * (base[2] & 3) : lx + 8 * ly;
}

template <int DIM>
__global__ __launch_bounds__(256) void k_tile_count2(Blocks B, int nb, int N, int64_t n_s,
                                                     const double* cp, const int* eflag,
                                                     const int* tile_blk_of, int* cnt2) {
  NODE_PROLOGUE(DIM);
  if (eflag[dof]) return;
  const int bb = tile_blk_of[dof];
  if (bb < 0) return;
  const V3 y = load_v(cp, n_s, dof, DIM);
  int base[3];
  double t[3];
  stencil_base<DIM>(y, N, B.p, base, t);
  atomicAdd(&cnt2[(int64_t)bb * 64 + local_base_code<DIM>(base)], 1);
}

template <int DIM>
__global__ __launch_bounds__(256) void k_tile_fill(Blocks B, int nb, int N, int64_t n_s,
                                                   const double* cp, const int* eflag,
                                                   const int* tile_blk_of, int* pos2, int ntr,
                                                   int* perm, double* frac64, float* frac32,
                                                   unsigned* lbase) {
  NODE_PROLOGUE(DIM);
  if (eflag[dof]) return;
  const int bb = tile_blk_of[dof];
  if (bb < 0) return;
  const V3 y = load_v(cp, n_s, dof, DIM);
  int base[3];
  double t[3];
  stencil_base<DIM>(y, N, B.p, base, t);
  const int pos = atomicAdd(&pos2[(int64_t)bb * 64 + local_base_code<DIM>(base)], 1);
  perm[pos] = dof;
  for (int a = 0; a < DIM; ++a) {
    frac64[(int64_t)a * ntr + pos] = t[a];
    frac32[(int64_t)a * ntr + pos] = (float)t[a];
  }
  const unsigned lx = base[0] & (G::BX - 1), ly = base[1] & (G::BX - 1),
                 lz = DIM == 3 ? (base[2] & (G::BX - 1)) : 0;
  lbase[pos] = lx | (ly << 8) | (lz << 16);
}

// Rows that share a tile and a stencil base land in their bucket in the
// order k_tile_fill's atomics gave them; sort each bucket by DOF so that the
// tile order (and with it the summation order of the transposed apply's
// run sums) is the same on every build.  Buckets hold a few rows (the nodes
// along one normal line), so one thread per bucket sorts by insertion.
template <int DIM>
__global__ void k_tile_sort_buckets(int64_t nbk, const int* cnt, const int* end, int ntr,
                                    int* perm, double* frac64, float* frac32) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nbk;
       k += (int64_t)gridDim.x * blockDim.x) {
  if (cnt[k] < 2) continue;
  const int e = end[k], s = e - cnt[k];
  for (int i = s + 1; i < e; ++i) {
    const int key = perm[i];
    double f64[3];
    float f32[3];
    for (int a = 0; a < DIM; ++a) {
      f64[a] = frac64[(int64_t)a * ntr + i];
      f32[a] = frac32[(int64_t)a * ntr + i];
    }
    int j = i - 1;
    while (j >= s && perm[j] > key) {
      perm[j + 1] = perm[j];
      for (int a = 0; a < DIM; ++a) {
        frac64[(int64_t)a * ntr + j + 1] = frac64[(int64_t)a * ntr + j];
        frac32[(int64_t)a * ntr + j + 1] = frac32[(int64_t)a * ntr + j];
      }
      --j;
    }
    perm[j + 1] = key;
    for (int a = 0; a < DIM; ++a) {
      frac64[(int64_t)a * ntr + j + 1] = f64[a];
      frac32[(int64_t)a * ntr + j + 1] = f32[a];
    }
  }
  }
}

__global__ void k_tile_compact(const int* cnt, const int* off, const int* tidx, int nb,
                               int* tile_blk, int* tile_start) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < nb && cnt[b] > 0) {
    tile_blk[tidx[b]] = b;
    tile_start[tidx[b]] = off[b];
  }
}

__global__ void k_nonzero(const int* in, int n, int* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = in[i] > 0 ? 1 : 0;
}

// Explicit interpolation rows of swapped PDE rows.
template <int DIM>
__global__ __launch_bounds__(256) void k_erow_pde(Blocks B, int nb, int N, int64_t n_s,
                                                  const double* cp, const int* row_c,
                                                  const int* alpha_of, const double* side_v,
                                                  const int* eflag, const int* eidx,
                                                  int* erow_id, int* ecol, double* ew,
                                                  float* ew32, int* ebase) {
  NODE_PROLOGUE(DIM);
  constexpr int NM = DIM == 3 ? 64 : 16;
  if (!eflag[dof]) return;
  const int r = eidx[dof];
  erow_id[r] = dof;
  const V3 y = load_v(cp, n_s, dof, DIM);
  int base[3];
  double t[3];
  stencil_base<DIM>(y, N, B.p, base, t);
  for (int a = 0; a < DIM; ++a) ebase[r * DIM + a] = base[a];
  double w[3][4];
  for (int a = 0; a < DIM; ++a) lagrange_p<double>(B.p, t[a], w[a]);
  const int bb = block_of<DIM>(B, base[0], base[1], base[2]);
  const int lx = base[0] & (G::BX - 1), ly = base[1] & (G::BX - 1),
            lz = DIM == 3 ? (base[2] & (G::BX - 1)) : 0;
  const int rc = row_c[dof];
  const V3 vi = load_v(side_v, n_s, dof, DIM);
  const int np = B.p + 1, nmp = DIM == 3 ? np * np * np : np * np;
  for (int o = 0; o < NM; ++o) {
    if (o >= nmp) {   // quadratic stencils fill the first (p+1)^d slots
      ecol[(int64_t)r * NM + o] = -1;
      ew[(int64_t)r * NM + o] = 0.0;
      ew32[(int64_t)r * NM + o] = 0.0f;
      continue;
    }
    const int a = o % np, b = (o / np) % np, c = o / (np * np);
    int j = node_dof<DIM>(B, bb, lx + a, ly + b, lz + c);
    if (row_c[j] == rc && alpha_of[j] >= 0 &&
        dot3<DIM>(vi, load_v(side_v, n_s, j, DIM)) < 0.0)
      j = alpha_of[j];
    const double wt = DIM == 3 ? (w[2][c] * w[1][b]) * w[0][a] : w[1][b] * w[0][a];
    ecol[(int64_t)r * NM + o] = j;
    ew[(int64_t)r * NM + o] = wt;
    ew32[(int64_t)r * NM + o] = (float)wt;
  }
}


// Explicit interpolation rows of BC DOFs (Sec. 4.3).  A BC DOF whose node
// lies on side s stands in for side -s, so it takes that side's condition.
//   Dirichlet, second order: u_alpha = 2 g - u(cpbar_C(x)), cpbar_C(x) =
//     cp_S(2 cp_C(x) - x) (eq. cpc-bar), weights -w, constant 2 g.
//   Dirichlet, first order: no linear part, constant g (u_alpha = g).
//   Zero Neumann: u_alpha = u(y) with y = cp_C(x) (first order, eq.
//     IBC-1st-order-Neumann) or cpbar_C(x) (second order), weights +w, no
//     constant.
// A member stays a BC DOF when it lies in Omega(C) on the director's side
// (d*_alpha = v of the node) and is the PDE DOF otherwise.  ecoef receives
// the multiplier of g in the row's constant (2, 1 or 0).
template <int DIM>
__global__ void k_erow_bc(Blocks B, int N, int64_t n_s, int64_t n_c, int order,
                          cpm_surface S, IBCList L, const int* bc_node, const double* bc_cpc,
                          const int* bc_side, const int* bc_curve, const int* bc_k,
                          const int* row_c, const int* alpha_of, const double* side_v, int r0,
                          int* erow_id, int* ecol, double* ew, float* ew32, int* ebase,
                          double* ecoef, unsigned long long* counters) {
  using G = Geo<DIM>;
  constexpr int NM = DIM == 3 ? 64 : 16;
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_c) return;
  const int r = r0 + (int)k;
  erow_id[r] = (int)(n_s + k);
  const int served = -bc_side[k];
  const bool neumann = L.c[bc_curve[k]].bc[served > 0 ? 0 : 1] == CPM_BC_NEUMANN;
  ecoef[k] = neumann ? 0.0 : (order == 2 ? 2.0 : 1.0);
  if (order != 2 && !neumann) {
    for (int o = 0; o < NM; ++o) {
      ecol[(int64_t)r * NM + o] = -1;
      ew[(int64_t)r * NM + o] = 0.0;
      ew32[(int64_t)r * NM + o] = 0.0f;
    }
    for (int a = 0; a < DIM; ++a) ebase[r * DIM + a] = 0;
    return;
  }
  const int j0 = bc_node[k];
  const V3 x = node_pos(bc_k[k * 3], bc_k[k * 3 + 1], bc_k[k * 3 + 2], N);
  const V3 pc{bc_cpc[k * DIM], bc_cpc[k * DIM + 1], DIM == 3 ? bc_cpc[k * DIM + 2] : 0.0};
  const V3 z{2.0 * pc.x - x.x, 2.0 * pc.y - x.y, DIM == 3 ? 2.0 * pc.z - x.z : 0.0};
  const V3 y = order == 2 ? cp_surface<DIM>(S, z) : pc;
  const double sgn = neumann ? 1.0 : -1.0;
  int base[3];
  double t[3];
  stencil_base<DIM>(y, N, B.p, base, t);
  for (int a = 0; a < DIM; ++a) ebase[r * DIM + a] = base[a];
  double w[3][4];
  for (int a = 0; a < DIM; ++a) lagrange_p<double>(B.p, t[a], w[a]);
  const int bb = block_of<DIM>(B, base[0], base[1], base[2]);
  const int lx = base[0] & (G::BX - 1), ly = base[1] & (G::BX - 1),
            lz = DIM == 3 ? (base[2] & (G::BX - 1)) : 0;
  const int rc = row_c[j0];
  const V3 vj = load_v(side_v, n_s, j0, DIM);
  int holes = 0;
  const int np = B.p + 1, nmp = DIM == 3 ? np * np * np : np * np;
  for (int o = 0; o < NM; ++o) {
    if (o >= nmp) {
      ecol[(int64_t)r * NM + o] = -1;
      ew[(int64_t)r * NM + o] = 0.0;
      ew32[(int64_t)r * NM + o] = 0.0f;
      continue;
    }
    const int a = o % np, b = (o / np) % np, c = o / (np * np);
    int m = bb < 0 ? -1 : node_dof<DIM>(B, bb, lx + a, ly + b, lz + c);
    if (m < 0) {
      ++holes;
    } else if (alpha_of[m] >= 0 && row_c[m] == rc &&
               !(dot3<DIM>(vj, load_v(side_v, n_s, m, DIM)) < 0.0)) {
      m = alpha_of[m];
    }
    const double wt = sgn * (DIM == 3 ? (w[2][c] * w[1][b]) * w[0][a] : w[1][b] * w[0][a]);
    ecol[(int64_t)r * NM + o] = m;
    ew[(int64_t)r * NM + o] = wt;
    ew32[(int64_t)r * NM + o] = (float)wt;
  }
  if (holes) atomicAdd(&counters[3], (unsigned long long)holes);
}

// FD neighbours of PDE rows in a check region: swap flag (eq.
// stencil-crossing-test applied to the FD stencil).
template <int DIM>
__global__ __launch_bounds__(256) void k_lflag(Blocks B, int nb, int64_t n_s, const int* row_c,
                                               const int* alpha_of, const double* side_v,
                                               int* lflag) {
  NODE_PROLOGUE(DIM);
  const int rc = row_c[dof];
  int sw = 0;
  if (rc >= 0) {
    const V3 vi = load_v(side_v, n_s, dof, DIM);
    const int l[3] = {G::lx(slot), G::ly(slot), G::lz(slot)};
    for (int f = 0; f < 2 * DIM; ++f) {
      int m[3] = {l[0], l[1], l[2]};
      m[f >> 1] += (f & 1) ? 1 : -1;
      const int k = node_dof<DIM>(B, blk, m[0], m[1], m[2]);
      if (k >= 0 && alpha_of[k] >= 0 && row_c[k] == rc &&
          dot3<DIM>(vi, load_v(side_v, n_s, k, DIM)) < 0.0)
        sw = 1;
    }
  }
  lflag[dof] = sw;
}

template <int DIM>
__global__ __launch_bounds__(256) void k_lrow_pde(Blocks B, int nb, int64_t n_s, const int* row_c,
                                                  const int* alpha_of, const double* side_v,
                                                  const int* lflag, const int* lidx,
                                                  int* lrow_id, int* lcol, int* lcol0,
                                                  unsigned long long* lrow_mask) {
  NODE_PROLOGUE(DIM);
  if (!lflag[dof]) return;
  const int r = lidx[dof];
  lrow_id[r] = dof;
  atomicOr(&lrow_mask[blk], 1ull << slot);
  const int rc = row_c[dof];
  const V3 vi = load_v(side_v, n_s, dof, DIM);
  const int l[3] = {G::lx(slot), G::ly(slot), G::lz(slot)};
  for (int f = 0; f < 2 * DIM; ++f) {
    int m[3] = {l[0], l[1], l[2]};
    m[f >> 1] += (f & 1) ? 1 : -1;
    const int k = node_dof<DIM>(B, blk, m[0], m[1], m[2]);
    int col = k;
    if (k >= 0 && alpha_of[k] >= 0 && row_c[k] == rc &&
        dot3<DIM>(vi, load_v(side_v, n_s, k, DIM)) < 0.0)
      col = alpha_of[k];
    lcol0[r * 2 * DIM + f] = k;
    lcol[r * 2 * DIM + f] = col;
  }
}

// FD rows of BC DOFs (eq. FD-crossing-test): neighbours outside Omega(C) are
// removed; a neighbour stays a BC DOF unless it lies on the other side.
template <int DIM>
__global__ void k_lrow_bc(Blocks B, int N, cpm_surface S, IBCList L, int64_t n_s, int64_t n_c,
                          const int* bc_node, const int* bc_k, const int* row_c,
                          const int* alpha_of, const double* side_v, int r0, int* lrow_id,
                          int* lcol, int* lcol0) {
  using G = Geo<DIM>;
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_c) return;
  const int r = r0 + (int)k;
  lrow_id[r] = (int)(n_s + k);
  const int j0 = bc_node[k];
  const int rc = row_c[j0];
  const V3 vj = load_v(side_v, n_s, j0, DIM);
  const int kk[3] = {bc_k[k * 3], bc_k[k * 3 + 1], bc_k[k * 3 + 2]};
  const int blk = block_of<DIM>(B, kk[0], kk[1], kk[2]);
  const int l[3] = {kk[0] & (G::BX - 1), kk[1] & (G::BX - 1), DIM == 3 ? (kk[2] & (G::BX - 1)) : 0};
  for (int f = 0; f < 2 * DIM; ++f) {
    int m[3] = {l[0], l[1], l[2]};
    m[f >> 1] += (f & 1) ? 1 : -1;
    const int q = node_dof<DIM>(B, blk, m[0], m[1], m[2]);
    int col = -1;
    if (q >= 0 && alpha_of[q] >= 0 && row_c[q] == rc) {
      col = dot3<DIM>(vj, load_v(side_v, n_s, q, DIM)) < 0.0 ? q : alpha_of[q];
    } else if (q >= 0) {
      // past the end of an open curve the solution is single valued: a
      // neighbour there without a BC DOF is its PDE DOF
      int qk[3] = {kk[0], kk[1], kk[2]};
      qk[f >> 1] += (f & 1) ? 1 : -1;
      if (curve_at_end(S, L.c[rc], node_pos(qk[0], qk[1], DIM == 3 ? qk[2] : 0, N))) col = q;
    }
    lcol0[r * 2 * DIM + f] = -1;
    lcol[r * 2 * DIM + f] = col;
  }
}

// Per-tile metadata of the staged blocks and per-block Laplacian metadata.
__global__ void k_tile_meta(Blocks B, int ntiles, int nq, int nnbr, const int* tile_blk,
                            QMeta* meta) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (int64_t)ntiles * 8) return;
  const int t = (int)(g >> 3), q = (int)(g & 7);
  QMeta m{0ull, 0, -1};
  if (q < nq) {
    const int qx = q & 1, qy = (q >> 1) & 1, qz = q >> 2;
    const int tb = tile_blk[t];
    const int code = nnbr == 27 ? (qz + 1) * 9 + (qy + 1) * 3 + (qx + 1) : (qy + 1) * 3 + (qx + 1);
    const int id = q == 0 ? tb : B.nbr[tb * nnbr + code];
    if (id >= 0) m = QMeta{B.mask[id], B.off[id], id};
  }
  meta[g] = m;
}

// Parity class of a tile's block: two tiles of one class stage disjoint
// sets of blocks (their block coordinates differ by at least 2 along some
// axis, and a tile stages its block and the next one along each axis).
__global__ void k_tile_colour(int ntiles, const int* tile_blk, const int4* coord, int* colour) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntiles) return;
  const int4 c = coord[tile_blk[t]];
  colour[t] = (c.x & 1) | ((c.y & 1) << 1) | ((c.z & 1) << 2);
}

__global__ void k_blk_face(Blocks B, int nb, int dim, int nnbr, const unsigned long long* lrow_mask,
                           QMeta* face) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (int64_t)nb * 8) return;
  const int i = (int)(g >> 3), k = (int)(g & 7);
  QMeta m{0ull, 0, -1};
  if (k == 7) {
    m.mask = lrow_mask[i];
    m.pad = 0;   // instance id (0 for a single band)
  } else if (k <= 2 * dim) {
    int id = i;
    if (k > 0) {
      const int f = k - 1, s1 = (f & 1) ? 1 : -1;
      const int dx = (f >> 1) == 0 ? s1 : 0, dy = (f >> 1) == 1 ? s1 : 0, dz = (f >> 1) == 2 ? s1 : 0;
      const int code = nnbr == 27 ? (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1) : (dy + 1) * 3 + (dx + 1);
      id = B.nbr[i * nnbr + code];
    }
    if (id >= 0) m = QMeta{B.mask[id], B.off[id], id};
  }
  face[g] = m;
}

// ---------------------------------------------------------------- export
template <int DIM>
__global__ __launch_bounds__(256) void k_export_rows(Blocks B, int nb, int N, int64_t n_s,
                                                     const double* cp, int* coords, int* ecols,
                                                     int* lcols, int* bases) {
  NODE_PROLOGUE(DIM);
  constexpr int NM = DIM == 3 ? 64 : 16;
  const int k3[3] = {kx, ky, kz};
  if (coords)
    for (int a = 0; a < DIM; ++a) coords[(int64_t)dof * DIM + a] = k3[a];
  if (ecols || bases) {
    const V3 y = load_v(cp, n_s, dof, DIM);
    int base[3];
    double t[3];
    stencil_base<DIM>(y, N, B.p, base, t);
    if (bases)
      for (int a = 0; a < DIM; ++a) bases[(int64_t)dof * DIM + a] = base[a];
    if (ecols) {
      const int bb = block_of<DIM>(B, base[0], base[1], base[2]);
      const int lx = base[0] & (G::BX - 1), ly = base[1] & (G::BX - 1),
                lz = DIM == 3 ? (base[2] & (G::BX - 1)) : 0;
      const int np = B.p + 1, nmp = DIM == 3 ? np * np * np : np * np;
      for (int o = 0; o < NM; ++o)
        ecols[(int64_t)dof * NM + o] =
            (bb < 0 || o >= nmp) ? -1
                                 : node_dof<DIM>(B, bb, lx + o % np, ly + (o / np) % np,
                                                 lz + o / (np * np));
    }
  }
  if (lcols) {
    const int l[3] = {G::lx(slot), G::ly(slot), G::lz(slot)};
    for (int f = 0; f < 2 * DIM; ++f) {
      int m[3] = {l[0], l[1], l[2]};
      m[f >> 1] += (f & 1) ? 1 : -1;
      lcols[(int64_t)dof * 2 * DIM + f] = node_dof<DIM>(B, blk, m[0], m[1], m[2]);
    }
  }
}

__global__ void k_export_erows(int n_erows, int nm, int dim, const int* erow_id, const int* ecol,
                               const int* ebase, int* ecols, int* bases) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n_erows * nm) return;
  const int r = (int)(t / nm), o = (int)(t % nm);
  const int id = erow_id[r];
  if (ecols) ecols[(int64_t)id * nm + o] = ecol[t];
  if (bases && o < dim) bases[(int64_t)id * dim + o] = ebase[r * dim + o];
}

__global__ void k_export_lrows(int n_lrows, int nf, const int* lrow_id, const int* lcol, int* lcols) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n_lrows * nf) return;
  const int r = (int)(t / nf), f = (int)(t % nf);
  lcols[(int64_t)lrow_id[r] * nf + f] = lcol[t];
}

// ================================================================== host
namespace {

Blocks view(const cpm_band* b) {
  return Blocks{b->blk_coord, b->blk_mask, b->blk_off, b->blk_nbr, b->hkeys, b->hvals, b->hcap,
                b->p};
}

// A temporary device buffer from a band's allocator, released at scope exit
// (only work on the stream that used it can still be queued: the builder and
// the export run on one stream).
template <class T>
struct Tmp {
  T* p = nullptr;
  size_t bytes = 0;
  const DevAlloc* da;
  Tmp(const cpm_band* owner, size_t n) : bytes((n ? n : 1) * sizeof(T)), da(&owner->da) {
    p = static_cast<T*>(da->get(bytes));
  }
  ~Tmp() { da->put(p, bytes); }
  Tmp(const Tmp&) = delete;
  Tmp& operator=(const Tmp&) = delete;
};

template <class T>
T read1(const T* d, hipStream_t s) {
  T h;
  CPM_HIP(hipMemcpyAsync(&h, d, sizeof(T), hipMemcpyDeviceToHost, s));
  CPM_HIP(hipStreamSynchronize(s));
  return h;
}

double reach_of(const cpm_surface& S) {
  if (S.kind == CPM_SURF_TORUS) return std::min(S.rho, S.R - S.rho);
  return S.R;
}

// ---- pull lists of the transposed explicit rows --------------------------
// The transposed apply adds every explicit row's contributions into their
// target entries.  Sorting (target, source) pairs once per band lets a pull
// kernel sum each target's contributions in a fixed order, with no atomics.
constexpr int kNoTarget = 0x7fffffff;

// E rows: entry g = i * nm + o targets ecol[g] (if a column)
__global__ void k_pull_pairs_e(int64_t ne, const int* ecol, int* key, int* val) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ne) return;
  const int c = ecol[g];
  key[g] = c >= 0 ? c : kNoTarget;
  val[g] = (int)g;
}

// L rows: entry (i, f, s) of explicit FD row i and neighbour f; a swapped
// PDE entry moves its contribution from the unswapped column k0 (s = 1,
// subtracted) to k1 (s = 0, added); a BC row adds to every column k1.
// val = 2 i + s.
__global__ void k_pull_pairs_l(int nrows, int nf, int64_t n_s, const int* row_id,
                               const int* lcol, const int* lcol0, int* key, int* val) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (int64_t)nrows * nf * 2) return;
  const int i = (int)(g / (2 * nf)), f = (int)((g / 2) % nf), sgn = (int)(g & 1);
  const int k1 = lcol[(int64_t)i * nf + f];
  int t = kNoTarget;
  if (row_id[i] < n_s) {
    const int k0 = lcol0[(int64_t)i * nf + f];
    if (k0 != k1) {
      if (sgn == 1 && k0 >= 0) t = k0;
      if (sgn == 0 && k1 >= 0) t = k1;
    }
  } else if (sgn == 0 && k1 >= 0) {
    t = k1;
  }
  key[g] = t;
  val[g] = 2 * i + sgn;
}

// E pull entries in sorted order: the source's weights (both precisions) and
// its row's DOF, which replaces the source index in place
__global__ void k_pull_denorm_e(int total, int* src, int nm, const int* erow_id, const double* ew,
                                const float* ew32, double* w64, float* w32) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int g = src[e];
  w64[e] = ew[g];
  w32[e] = ew32[g];
  src[e] = erow_id[g / nm];
}

// Sorts the pairs by target (stable: sources ascending within a target) and
// stores the distinct targets, their segment starts and the sources.
static void build_pull(cpm_band* b, int64_t ne, Tmp<int>& key, Tmp<int>& val, hipStream_t st,
                       int& n_tgt, int*& tgt, int*& start, int*& src) {
  n_tgt = 0;
  if (ne <= 0) return;
  if (ne >= (1ll << 31)) CPM_FAIL(CPM_E_INVALID, "too many explicit-row entries");
  const int n = (int)ne;
  Tmp<int> key2(b, n), val2(b, n), uniq(b, n), cnt(b, n), nrun(b, 1);
  size_t tb = 0;
  CPM_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tb, key.p, key2.p, val.p, val2.p, n, 0, 31, st));
  {
    Tmp<unsigned char> tmp(b, tb);
    CPM_HIP(hipcub::DeviceRadixSort::SortPairs(tmp.p, tb, key.p, key2.p, val.p, val2.p, n, 0, 31,
                                               st));
  }
  tb = 0;
  CPM_HIP(hipcub::DeviceRunLengthEncode::Encode(nullptr, tb, key2.p, uniq.p, cnt.p, nrun.p, n, st));
  {
    Tmp<unsigned char> tmp(b, tb);
    CPM_HIP(hipcub::DeviceRunLengthEncode::Encode(tmp.p, tb, key2.p, uniq.p, cnt.p, nrun.p, n, st));
  }
  int runs = 0;
  CPM_HIP(hipMemcpyAsync(&runs, nrun.p, sizeof(int), hipMemcpyDeviceToHost, st));
  CPM_HIP(hipStreamSynchronize(st));
  std::vector<int> hu(runs), hc(runs);
  CPM_HIP(hipMemcpyAsync(hu.data(), uniq.p, sizeof(int) * runs, hipMemcpyDeviceToHost, st));
  CPM_HIP(hipMemcpyAsync(hc.data(), cnt.p, sizeof(int) * runs, hipMemcpyDeviceToHost, st));
  CPM_HIP(hipStreamSynchronize(st));
  int nt = runs;
  if (nt && hu[nt - 1] == kNoTarget) --nt;   // entries without a target sort last
  std::vector<int> hs(nt + 1, 0);
  for (int k = 0; k < nt; ++k) hs[k + 1] = hs[k] + hc[k];
  n_tgt = nt;
  tgt = b->alloc<int>(nt);
  start = b->alloc<int>(nt + 1);
  src = b->alloc<int>(hs[nt]);
  if (nt) {
    CPM_HIP(hipMemcpyAsync(tgt, hu.data(), sizeof(int) * nt, hipMemcpyHostToDevice, st));
    CPM_HIP(hipMemcpyAsync(start, hs.data(), sizeof(int) * (nt + 1), hipMemcpyHostToDevice, st));
    CPM_HIP(hipMemcpyAsync(src, val2.p, sizeof(int) * hs[nt], hipMemcpyDeviceToDevice, st));
  }
  CPM_HIP(hipStreamSynchronize(st));
}

// ---- stencil set (Sec. 5.1), marked on a built tube band --------------
// flag[id] = 1 for every row id of a list
__global__ void k_ss_flag(const int* ids, int n, unsigned char* flag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) flag[ids[i]] = 1;
}

// used[j] = 1 for every member j of the stencil of a PDE row whose E row is
// not explicit (an explicit row's columns are marked by k_ss_cols)
template <int DIM>
__global__ __launch_bounds__(256) void k_ss_members(Blocks B, int nb, int N, int64_t n_s,
                                                    const double* cp, const unsigned char* isE,
                                                    unsigned char* used) {
  NODE_PROLOGUE(DIM);
  if (isE[dof]) return;
  const V3 y = load_v(cp, n_s, dof, DIM);
  int base[3];
  double t[3];
  stencil_base<DIM>(y, N, B.p, base, t);
  const int bb = block_of<DIM>(B, base[0], base[1], base[2]);
  if (bb < 0) return;
  const int lx = base[0] & (G::BX - 1), ly = base[1] & (G::BX - 1),
            lz = DIM == 3 ? (base[2] & (G::BX - 1)) : 0;
  const int np = B.p + 1, nmp = DIM == 3 ? np * np * np : np * np;
  for (int o = 0; o < nmp; ++o) {
    const int a = o % np, bq = (o / np) % np, c = o / (np * np);
    const int j = node_dof<DIM>(B, bb, lx + a, ly + bq, lz + c);
    if (j >= 0) used[j] = 1;
  }
}

// flag[c] = 1 for every stored column c >= 0 of a [nrows][w] column table,
// restricted to rows whose id is flagged in `only` (null: every row)
__global__ void k_ss_cols(const int* ids, const int* col, int nrows, int w,
                          const unsigned char* only, unsigned char* flag) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (int64_t)nrows * w) return;
  const int i = (int)(g / w);
  if (only && !only[ids[i]]) return;
  const int c = col[g];
  if (c >= 0) flag[c] = 1;
}

// need[j] = 1 for every used PDE row and its face neighbours in the band,
// for rows whose FD stencil is not explicit (those go through k_ss_cols)
template <int DIM>
__global__ __launch_bounds__(256) void k_ss_fd(Blocks B, int nb, const unsigned char* used,
                                               const unsigned char* isL, unsigned char* need) {
  NODE_PROLOGUE(DIM);
  if (!used[dof]) return;
  need[dof] = 1;
  if (isL[dof]) return;
  const int l[3] = {G::lx(slot), G::ly(slot), G::lz(slot)};
  for (int f = 0; f < 2 * DIM; ++f) {
    int q[3] = {l[0], l[1], l[2]};
    q[f >> 1] += (f & 1) ? 1 : -1;
    const int j = node_dof<DIM>(B, blk, q[0], q[1], q[2]);
    if (j >= 0) need[j] = 1;
  }
}

// a needed BC DOF keeps its node; need[] over BC DOFs is also set for used
// BC rows (their own index)
__global__ void k_ss_bcnodes(int64_t n_s, int64_t n_c, const int* bc_node,
                             const unsigned char* used, unsigned char* need) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_c) return;
  if (used[n_s + k]) need[n_s + k] = 1;
  if (need[n_s + k] || used[n_s + k]) need[bc_node[k]] = 1;
}

// keep[blk] = the block's slots whose PDE DOF is needed
__global__ void k_ss_masks(const unsigned long long* mask, const int* off, int nb,
                           const unsigned char* need, unsigned long long* keep) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  const unsigned long long m = mask[b];
  unsigned long long k = 0ull;
  int d = off[b];
  for (int s2 = 0; s2 < 64; ++s2)
    if ((m >> s2) & 1ull) {
      if (need[d]) k |= 1ull << s2;
      ++d;
    }
  keep[b] = k;
}

template <int DIM>
void build(cpm_band* b, hipStream_t st, const Filter& F);

// The stencil set of a built tube band t: per block of t, the nodes that
// carry a column of E (a member of some interpolation stencil) or an FD
// neighbour of such a DOF's row, or the node of a BC DOF of either kind.
// keep must hold t->nb entries; the filter refers to t's hash table.
template <int DIM>
Filter stencil_set_filter(const cpm_band* t, hipStream_t st, unsigned long long* keep) {
  const int64_t n = t->n, n_s = t->n_s;
  const int nm = DIM == 3 ? 64 : 16;
  Tmp<unsigned char> isE(t, n), isL(t, n), used(t, n), need(t, n);
  CPM_HIP(hipMemsetAsync(isE.p, 0, n, st));
  CPM_HIP(hipMemsetAsync(isL.p, 0, n, st));
  CPM_HIP(hipMemsetAsync(used.p, 0, n, st));
  CPM_HIP(hipMemsetAsync(need.p, 0, n, st));
  const Blocks B = view(t);
  const dim3 gnode((t->nb + 3) / 4);
  if (t->n_erows)
    hipLaunchKernelGGL(k_ss_flag, dim3(grid_for(t->n_erows, 256)), dim3(256), 0, st, t->erow_id,
                       t->n_erows, isE.p);
  if (t->n_lrows)
    hipLaunchKernelGGL(k_ss_flag, dim3(grid_for(t->n_lrows, 256)), dim3(256), 0, st, t->lrow_id,
                       t->n_lrows, isL.p);
  hipLaunchKernelGGL(k_ss_members<DIM>, gnode, dim3(256), 0, st, B, t->nb, t->N, n_s, t->cp,
                     isE.p, used.p);
  if (t->n_erows)
    hipLaunchKernelGGL(k_ss_cols, dim3(grid_for((int64_t)t->n_erows * nm, 256)), dim3(256), 0, st,
                       t->erow_id, t->ecol, t->n_erows, nm, nullptr, used.p);
  hipLaunchKernelGGL(k_ss_fd<DIM>, gnode, dim3(256), 0, st, B, t->nb, used.p, isL.p, need.p);
  if (t->n_lrows)
    hipLaunchKernelGGL(k_ss_cols, dim3(grid_for((int64_t)t->n_lrows * 2 * DIM, 256)), dim3(256), 0,
                       st, t->lrow_id, t->lcol, t->n_lrows, 2 * DIM, used.p, need.p);
  if (t->n_c)
    hipLaunchKernelGGL(k_ss_bcnodes, dim3(grid_for(t->n_c, 256)), dim3(256), 0, st, n_s, t->n_c,
                       t->bc_node, used.p, need.p);
  hipLaunchKernelGGL(k_ss_masks, dim3(grid_for(t->nb, 256)), dim3(256), 0, st, t->blk_mask,
                     t->blk_off, t->nb, need.p, keep);
  CPM_LAUNCH_CHECK();
  CPM_HIP(hipStreamSynchronize(st));
  Filter F;
  F.hkeys = t->hkeys;
  F.hvals = t->hvals;
  F.hcap = t->hcap;
  F.keep = keep;
  return F;
}

template <int DIM>
void build(cpm_band* b, hipStream_t st, const Filter& F) {
  using G = Geo<DIM>;
  const cpm_surface& S = b->surf;
  const int N = b->N;
  const double r = b->r;

  // ---- bounding box of blocks
  double ext[3] = {S.R, S.R, S.R};
  if (S.kind == CPM_SURF_TORUS) {
    ext[0] = ext[1] = S.R + S.rho;
    ext[2] = S.rho;
  }
  Box box{};
  for (int a = 0; a < 3; ++a) {
    if (a >= DIM) {
      box.blo[a] = 0;
      box.nb[a] = 1;
      continue;
    }
    const long lo = (long)std::floor((S.center[a] - ext[a] - r) * N) - 2;
    const long hi = (long)std::ceil((S.center[a] + ext[a] + r) * N) + 2;
    const long blo = lo >> G::SH, bhi = hi >> G::SH;
    box.blo[a] = (int)blo;
    box.nb[a] = (int)(bhi - blo + 1);
  }
  const int64_t nrows = (int64_t)box.nb[1] * box.nb[2];
  const double half_diag = 0.5 * (G::BX - 1) * std::sqrt((double)DIM);
  const double thr = r + (half_diag + 0.01) / N;

  // ---- pass 1: occupied blocks (row by row), then sorted into Morton order
  Tmp<int> row_count(b, nrows), row_off(b, nrows);
  hipLaunchKernelGGL((k_classify<DIM, false>), dim3(nrows), dim3(256), 0, st, S, N, r, thr, box,
                     row_count.p, nullptr, nullptr, nullptr, F);
  CPM_LAUNCH_CHECK();
  const int64_t nb64 = scan_exclusive_i32(row_count.p, row_off.p, nrows, st, b->da);
  if (nb64 <= 0) CPM_FAIL(CPM_E_INVALID, "the band is empty (N = %d)", N);
  if (nb64 > (1 << 27)) CPM_FAIL(CPM_E_INVALID, "band too large: %lld blocks", (long long)nb64);
  const int nb = (int)nb64;
  b->nb = nb;
  b->blk_coord = b->alloc<int4>(nb);
  b->blk_mask = b->alloc<unsigned long long>(nb);
  b->blk_off = b->alloc<int>(nb + 1);
  {
    Tmp<int4> coord0(b, nb);
    Tmp<unsigned long long> mask0(b, nb), key0(b, nb), key1(b, nb);
    Tmp<int> idx0(b, nb), idx1(b, nb);
    hipLaunchKernelGGL((k_classify<DIM, true>), dim3(nrows), dim3(256), 0, st, S, N, r, thr, box,
                       nullptr, row_off.p, coord0.p, mask0.p, F);
    CPM_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_morton, dim3(grid_for(nb, 256)), dim3(256), 0, st, coord0.p, nb, key0.p,
                       idx0.p);
    CPM_LAUNCH_CHECK();
    size_t tb = 0;
    CPM_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tb, key0.p, key1.p, idx0.p, idx1.p, nb, 0,
                                               63, st));
    Tmp<unsigned char> tmp(b, tb);
    CPM_HIP(hipcub::DeviceRadixSort::SortPairs(tmp.p, tb, key0.p, key1.p, idx0.p, idx1.p, nb, 0,
                                               63, st));
    hipLaunchKernelGGL(k_permute_blocks, dim3(grid_for(nb, 256)), dim3(256), 0, st, idx1.p, nb,
                       coord0.p, mask0.p, b->blk_coord, b->blk_mask);
    CPM_LAUNCH_CHECK();
    CPM_HIP(hipStreamSynchronize(st));
  }
  {
    Tmp<int> cnt(b, nb);
    hipLaunchKernelGGL(k_popcounts, dim3(grid_for(nb, 256)), dim3(256), 0, st, b->blk_mask, nb, cnt.p);
    CPM_LAUNCH_CHECK();
    b->n_s = scan_exclusive_i32(cnt.p, b->blk_off, nb, st, b->da);
    const int ns32 = (int)b->n_s;
    CPM_HIP(hipMemcpyAsync(b->blk_off + nb, &ns32, sizeof(int), hipMemcpyHostToDevice, st));
    CPM_HIP(hipStreamSynchronize(st));
  }
  if (b->n_s >= (1ll << 30)) CPM_FAIL(CPM_E_INVALID, "band too large: %lld nodes", (long long)b->n_s);
  const int64_t n_s = b->n_s;

  // ---- hash table and neighbour table
  unsigned cap = 1024;
  while (cap < 2u * (unsigned)nb) cap <<= 1;
  b->hcap = cap;
  b->hkeys = b->alloc<unsigned long long>(cap);
  b->hvals = b->alloc<int>(cap);
  CPM_HIP(hipMemsetAsync(b->hkeys, 0xff, (size_t)cap * sizeof(unsigned long long), st));
  hipLaunchKernelGGL(k_hash_insert, dim3(grid_for(nb, 256)), dim3(256), 0, st, b->blk_coord, nb,
                     b->hkeys, b->hvals, cap);
  CPM_LAUNCH_CHECK();
  b->blk_nbr = b->alloc<int>((size_t)nb * G::NNBR);
  hipLaunchKernelGGL(k_neighbours<DIM>, dim3(grid_for((int64_t)nb * G::NNBR, 256)), dim3(256), 0, st,
                     view(b), nb, b->blk_nbr);
  CPM_LAUNCH_CHECK();
  const Blocks B = view(b);
  const dim3 gnode((nb + 3) / 4);

  // ---- stored closest points
  b->cp = b->alloc<double>((size_t)DIM * n_s);
  hipLaunchKernelGGL(k_rows<DIM>, gnode, dim3(256), 0, st, B, nb, S, N, n_s, b->cp);
  CPM_LAUNCH_CHECK();

  // ---- interior boundaries
  Tmp<unsigned long long> counters(b, 8);
  CPM_HIP(hipMemsetAsync(counters.p, 0, 8 * sizeof(unsigned long long), st));
  IBCList L{};
  L.n = b->n_ibc;
  for (int c = 0; c < b->n_ibc; ++c) L.c[c] = b->ibcs[c];
  const int nib = b->n_ibc;
  Tmp<int> row_c(b, nib ? n_s : 1), omega(b, nib ? n_s : 1), alpha_of(b, nib ? n_s : 1);
  Tmp<double> side_v(b, nib ? (size_t)DIM * n_s : 1), cpcs(b, nib ? (size_t)DIM * n_s : 1);
  std::unique_ptr<Tmp<int>> bc_kp;
  std::vector<int64_t> curve_count(nib, 0);
  if (nib) {
    hipLaunchKernelGGL(k_ibc_rows<DIM>, gnode, dim3(256), 0, st, B, nb, S, L, N, n_s, r,
                       b->check_factor, b->tau, b->cp, row_c.p, omega.p, side_v.p, cpcs.p,
                       counters.p);
    CPM_LAUNCH_CHECK();
    unsigned long long hc[4];
    CPM_HIP(hipMemcpyAsync(hc, counters.p, sizeof(hc), hipMemcpyDeviceToHost, st));
    CPM_HIP(hipStreamSynchronize(st));
    if (hc[2]) CPM_FAIL(CPM_E_OVERLAP, "the check regions of two interior boundaries overlap");
    b->on_c_nodes = (int64_t)hc[0];
    CPM_HIP(hipMemsetAsync(alpha_of.p, 0xff, n_s * sizeof(int), st));
    Tmp<int> flag(b, n_s), rank(b, n_s);
    for (int c = 0; c < nib; ++c) {
      hipLaunchKernelGGL(k_flag_curve, dim3(grid_for(n_s, 256)), dim3(256), 0, st, row_c.p,
                         omega.p, n_s, c, flag.p);
      CPM_LAUNCH_CHECK();
      curve_count[c] = scan_exclusive_i32(flag.p, rank.p, n_s, st, b->da);
      b->n_c += curve_count[c];
    }
    b->bc_node = b->alloc<int>(b->n_c);
    b->bc_cpc = b->alloc<double>((size_t)b->n_c * DIM);
    b->bc_side = b->alloc<int>(b->n_c);
    b->bc_curve = b->alloc<int>(b->n_c);
    bc_kp.reset(new Tmp<int>(b, (size_t)b->n_c * 3));
    int64_t base_alpha = 0;
    for (int c = 0; c < nib; ++c) {
      hipLaunchKernelGGL(k_flag_curve, dim3(grid_for(n_s, 256)), dim3(256), 0, st, row_c.p,
                         omega.p, n_s, c, flag.p);
      CPM_LAUNCH_CHECK();
      scan_exclusive_i32(flag.p, rank.p, n_s, st, b->da);
      hipLaunchKernelGGL(k_bc_assign<DIM>, gnode, dim3(256), 0, st, B, nb, flag.p, rank.p, n_s,
                         base_alpha, c, S, L, side_v.p, cpcs.p, alpha_of.p, b->bc_node,
                         b->bc_cpc, b->bc_side, b->bc_curve, bc_kp->p);
      CPM_LAUNCH_CHECK();
      base_alpha += curve_count[c];
    }
  }
  b->n = b->n_s + b->n_c;
  if (b->n >= (1ll << 30)) CPM_FAIL(CPM_E_INVALID, "system too large");
  const int64_t n_c = b->n_c;

  // ---- interpolation stencils: holes, swaps, tiles
  Tmp<int> eflag(b, n_s), tile_blk_of(b, n_s), tile_cnt(b, nb), tile_off(b, nb);
  CPM_HIP(hipMemsetAsync(tile_cnt.p, 0, nb * sizeof(int), st));
  hipLaunchKernelGGL(k_stencil_scan<DIM>, gnode, dim3(256), 0, st, B, nb, N, n_s, b->cp,
                     nib ? row_c.p : nullptr, alpha_of.p, side_v.p, eflag.p, tile_blk_of.p,
                     tile_cnt.p, counters.p);
  CPM_LAUNCH_CHECK();
  {
    unsigned long long hc[4];
    CPM_HIP(hipMemcpyAsync(hc, counters.p, sizeof(hc), hipMemcpyDeviceToHost, st));
    CPM_HIP(hipStreamSynchronize(st));
    if (hc[3])
      CPM_FAIL(CPM_E_STENCIL_HOLE, "%llu interpolation-stencil members are not band nodes "
               "(band radius %.6g = %.4g h too small for the interpolation stencils)",
               hc[3], r, r * N);
    b->no_bc_dof_swaps = (int64_t)hc[1];
  }
  // explicit E rows: swapped PDE rows then all BC rows
  constexpr int NM = DIM == 3 ? 64 : 16;
  {
    Tmp<int> eidx(b, n_s);
    const int64_t ne_pde = scan_exclusive_i32(eflag.p, eidx.p, n_s, st, b->da);
    b->n_erows = (int)(ne_pde + n_c);
    b->erow_id = b->alloc<int>(b->n_erows);
    b->ecol = b->alloc<int>((size_t)b->n_erows * NM);
    b->ew = b->alloc<double>((size_t)b->n_erows * NM);
    b->ew32 = b->alloc<float>((size_t)b->n_erows * NM);
    b->ebase = b->alloc<int>((size_t)b->n_erows * DIM);
    if (ne_pde)
      hipLaunchKernelGGL(k_erow_pde<DIM>, gnode, dim3(256), 0, st, B, nb, N, n_s, b->cp, row_c.p,
                         alpha_of.p, side_v.p, eflag.p, eidx.p, b->erow_id, b->ecol, b->ew,
                         b->ew32, b->ebase);
    CPM_LAUNCH_CHECK();
    b->bc_ecoef = b->alloc<double>(n_c);
    if (n_c)
      hipLaunchKernelGGL(k_erow_bc<DIM>, dim3(grid_for(n_c, 128)), dim3(128), 0, st, B, N, n_s,
                         n_c, b->order, S, L, b->bc_node, b->bc_cpc, b->bc_side, b->bc_curve,
                         bc_kp->p, row_c.p, alpha_of.p, side_v.p, (int)ne_pde, b->erow_id,
                         b->ecol, b->ew, b->ew32, b->ebase, b->bc_ecoef, counters.p);
    CPM_LAUNCH_CHECK();
    unsigned long long hc[4];
    CPM_HIP(hipMemcpyAsync(hc, counters.p, sizeof(hc), hipMemcpyDeviceToHost, st));
    CPM_HIP(hipStreamSynchronize(st));
    if (hc[3])
      CPM_FAIL(CPM_E_STENCIL_HOLE, "%llu mirror-stencil members are not band nodes", hc[3]);
  }
  // gather tiles
  {
    b->n_tile_rows = (int)scan_exclusive_i32(tile_cnt.p, tile_off.p, nb, st, b->da);
    Tmp<int> nz(b, nb), tidx(b, nb);
    hipLaunchKernelGGL(k_nonzero, dim3(grid_for(nb, 256)), dim3(256), 0, st, tile_cnt.p, nb, nz.p);
    CPM_LAUNCH_CHECK();
    b->ntiles = (int)scan_exclusive_i32(nz.p, tidx.p, nb, st, b->da);
    b->tile_blk = b->alloc<int>(b->ntiles);
    b->tile_start = b->alloc<int>(b->ntiles + 1);
    hipLaunchKernelGGL(k_tile_compact, dim3(grid_for(nb, 256)), dim3(256), 0, st, tile_cnt.p,
                       tile_off.p, tidx.p, nb, b->tile_blk, b->tile_start);
    CPM_LAUNCH_CHECK();
    CPM_HIP(hipMemcpyAsync(b->tile_start + b->ntiles, &b->n_tile_rows, sizeof(int),
                           hipMemcpyHostToDevice, st));
    const int ntr = b->n_tile_rows;
    b->perm = b->alloc<int>(ntr);
    b->frac64 = b->alloc<double>((size_t)DIM * ntr);
    b->frac32 = b->alloc<float>((size_t)DIM * ntr);
    b->lbase = b->alloc<unsigned>(ntr);
    {
      Tmp<int> cnt2(b, (size_t)nb * 64), pos2(b, (size_t)nb * 64);
      CPM_HIP(hipMemsetAsync(cnt2.p, 0, (size_t)nb * 64 * sizeof(int), st));
      hipLaunchKernelGGL(k_tile_count2<DIM>, gnode, dim3(256), 0, st, B, nb, N, n_s, b->cp,
                         eflag.p, tile_blk_of.p, cnt2.p);
      CPM_LAUNCH_CHECK();
      const int64_t tot = scan_exclusive_i32(cnt2.p, pos2.p, (int64_t)nb * 64, st, b->da);
      if (tot != ntr) CPM_FAIL(CPM_E_INVALID, "internal: tile row count mismatch");
      hipLaunchKernelGGL(k_tile_fill<DIM>, gnode, dim3(256), 0, st, B, nb, N, n_s, b->cp,
                         eflag.p, tile_blk_of.p, pos2.p, ntr, b->perm, b->frac64, b->frac32,
                         b->lbase);
      CPM_LAUNCH_CHECK();
      hipLaunchKernelGGL(k_tile_sort_buckets<DIM>, dim3(grid_for((int64_t)nb * 64, 256)),
                         dim3(256), 0, st, (int64_t)nb * 64, cnt2.p, pos2.p, ntr, b->perm,
                         b->frac64, b->frac32);
      CPM_LAUNCH_CHECK();
      CPM_HIP(hipStreamSynchronize(st));
    }
    CPM_LAUNCH_CHECK();
  }
  // explicit L rows: swapped PDE rows then all BC rows
  b->lrow_mask = b->alloc<unsigned long long>(nb);
  CPM_HIP(hipMemsetAsync(b->lrow_mask, 0, nb * sizeof(unsigned long long), st));
  {
    int64_t nl_pde = 0;
    Tmp<int> lflag(b, nib ? n_s : 1), lidx(b, nib ? n_s : 1);
    if (nib) {
      hipLaunchKernelGGL(k_lflag<DIM>, gnode, dim3(256), 0, st, B, nb, n_s, row_c.p, alpha_of.p,
                         side_v.p, lflag.p);
      CPM_LAUNCH_CHECK();
      nl_pde = scan_exclusive_i32(lflag.p, lidx.p, n_s, st, b->da);
    }
    b->n_lrows = (int)(nl_pde + n_c);
    b->lrow_id = b->alloc<int>(b->n_lrows);
    b->lcol = b->alloc<int>((size_t)b->n_lrows * 2 * DIM);
    b->lcol0 = b->alloc<int>((size_t)b->n_lrows * 2 * DIM);
    if (nl_pde)
      hipLaunchKernelGGL(k_lrow_pde<DIM>, gnode, dim3(256), 0, st, B, nb, n_s, row_c.p,
                         alpha_of.p, side_v.p, lflag.p, lidx.p, b->lrow_id, b->lcol, b->lcol0,
                         b->lrow_mask);
    CPM_LAUNCH_CHECK();
    if (n_c)
      hipLaunchKernelGGL(k_lrow_bc<DIM>, dim3(grid_for(n_c, 128)), dim3(128), 0, st, B, N, S, L,
                         n_s, n_c, b->bc_node, bc_kp->p, row_c.p, alpha_of.p, side_v.p,
                         (int)nl_pde, b->lrow_id, b->lcol, b->lcol0);
    CPM_LAUNCH_CHECK();
  }
  // pull lists of the transposed explicit rows
  {
    const int64_t ne = (int64_t)b->n_erows * NM;
    Tmp<int> key(b, ne ? ne : 1), val(b, ne ? ne : 1);
    if (ne) {
      hipLaunchKernelGGL(k_pull_pairs_e, dim3(grid_for(ne, 256)), dim3(256), 0, st, ne, b->ecol,
                         key.p, val.p);
      CPM_LAUNCH_CHECK();
    }
    build_pull(b, ne, key, val, st, b->n_et, b->et_tgt, b->et_start, b->et_src);
    if (b->n_et) {
      int total = 0;
      CPM_HIP(hipMemcpyAsync(&total, b->et_start + b->n_et, sizeof(int), hipMemcpyDeviceToHost, st));
      CPM_HIP(hipStreamSynchronize(st));
      b->n_et_entries = total;
      b->et_w = b->alloc<double>(total);
      b->et_w32 = b->alloc<float>(total);
      hipLaunchKernelGGL(k_pull_denorm_e, dim3(grid_for(total, 256)), dim3(256), 0, st, total,
                         b->et_src, NM, b->erow_id, b->ew, b->ew32, b->et_w, b->et_w32);
      CPM_LAUNCH_CHECK();
    }
    const int64_t nl = (int64_t)b->n_lrows * 2 * DIM * 2;
    Tmp<int> keyl(b, nl ? nl : 1), vall(b, nl ? nl : 1);
    if (nl) {
      hipLaunchKernelGGL(k_pull_pairs_l, dim3(grid_for(nl, 256)), dim3(256), 0, st, b->n_lrows,
                         2 * DIM, n_s, b->lrow_id, b->lcol, b->lcol0, keyl.p, vall.p);
      CPM_LAUNCH_CHECK();
    }
    build_pull(b, nl, keyl, vall, st, b->n_lt, b->lt_tgt, b->lt_start, b->lt_src);
  }
  // metadata read by the apply kernels
  b->tile_meta = b->alloc<QMeta>((size_t)b->ntiles * 8);
  if (b->ntiles)
    hipLaunchKernelGGL(k_tile_meta, dim3(grid_for((int64_t)b->ntiles * 8, 256)), dim3(256), 0, st,
                       B, b->ntiles, 1 << DIM, G::NNBR, b->tile_blk, b->tile_meta);
  CPM_LAUNCH_CHECK();
  // transpose schedule: tiles grouped by parity class (stable in tile order)
  b->tile_col = b->alloc<int4>(b->ntiles);
  std::fill(b->col_start, b->col_start + 9, 0);
  if (b->ntiles) {
    Tmp<int> colour(b, b->ntiles);
    hipLaunchKernelGGL(k_tile_colour, dim3(grid_for(b->ntiles, 256)), dim3(256), 0, st, b->ntiles,
                       b->tile_blk, b->blk_coord, colour.p);
    CPM_LAUNCH_CHECK();
    std::vector<int> hcol(b->ntiles), hstart(b->ntiles + 1);
    std::vector<int4> order(b->ntiles);
    CPM_HIP(hipMemcpyAsync(hcol.data(), colour.p, sizeof(int) * b->ntiles, hipMemcpyDeviceToHost,
                           st));
    CPM_HIP(hipMemcpyAsync(hstart.data(), b->tile_start, sizeof(int) * (b->ntiles + 1),
                           hipMemcpyDeviceToHost, st));
    CPM_HIP(hipStreamSynchronize(st));
    for (int t = 0; t < b->ntiles; ++t) ++b->col_start[hcol[t] + 1];
    for (int k = 0; k < 8; ++k) b->col_start[k + 1] += b->col_start[k];
    int next[8];
    std::copy(b->col_start, b->col_start + 8, next);
    for (int t = 0; t < b->ntiles; ++t)
      order[next[hcol[t]]++] = make_int4(t, hstart[t], hstart[t + 1], 0);
    CPM_HIP(hipMemcpyAsync(b->tile_col, order.data(), sizeof(int4) * b->ntiles,
                           hipMemcpyHostToDevice, st));
    CPM_HIP(hipStreamSynchronize(st));
  }
  b->blk_face = b->alloc<QMeta>((size_t)nb * 8);
  hipLaunchKernelGGL(k_blk_face, dim3(grid_for((int64_t)nb * 8, 256)), dim3(256), 0, st, B, nb,
                     DIM, G::NNBR, b->lrow_mask, b->blk_face);
  CPM_LAUNCH_CHECK();
  CPM_HIP(hipStreamSynchronize(st));
}

template <int DIM>
void export_rows(const cpm_band* b, int* coords, int* ecols, int* lcols, int* bases,
                 hipStream_t st) {
  const dim3 gnode((b->nb + 3) / 4);
  hipLaunchKernelGGL(k_export_rows<DIM>, gnode, dim3(256), 0, st, view(b), b->nb, b->N, b->n_s,
                     b->cp, coords, ecols, lcols, bases);
  CPM_LAUNCH_CHECK();
  const int nm = DIM == 3 ? 64 : 16;
  if ((ecols || bases) && b->n_erows)
    hipLaunchKernelGGL(k_export_erows, dim3(grid_for((int64_t)b->n_erows * nm, 256)), dim3(256),
                       0, st, b->n_erows, nm, DIM, b->erow_id, b->ecol, b->ebase, ecols, bases);
  CPM_LAUNCH_CHECK();
  if (lcols && b->n_lrows)
    hipLaunchKernelGGL(k_export_lrows, dim3(grid_for((int64_t)b->n_lrows * 2 * DIM, 256)),
                       dim3(256), 0, st, b->n_lrows, 2 * DIM, b->lrow_id, b->lcol, lcols);
  CPM_LAUNCH_CHECK();
}

}  // namespace
}  // namespace cpm

using namespace cpm;

extern "C" cpm_status cpm_build_band(const cpm_surface* surface, const cpm_ibc* ibcs, int n_ibc,
                                     const cpm_grid* grid, const cpm_allocator* allocator,
                                     void* hip_stream, cpm_band** out) {
  return guard([&] {
    if (!surface || !grid || !out) CPM_FAIL(CPM_E_INVALID, "null argument");
    if (allocator && (!allocator->alloc || !allocator->free))
      CPM_FAIL(CPM_E_INVALID, "an allocator needs both alloc and free");
    *out = nullptr;
    if (grid->N <= 0) CPM_FAIL(CPM_E_INVALID, "N must be positive (got %d)", grid->N);
    if (grid->p != 3 && grid->p != 2)
      CPM_FAIL(CPM_E_INVALID, "interpolation degree p must be 2 or 3 (got %d)", grid->p);
    if (grid->order != 1 && grid->order != 2)
      CPM_FAIL(CPM_E_INVALID, "order must be 1 or 2 (got %d)", grid->order);
    if (n_ibc < 0 || n_ibc > kMaxIBC || (n_ibc && !ibcs))
      CPM_FAIL(CPM_E_INVALID, "n_ibc must be in [0, %d] with a non-null array", kMaxIBC);
    const int kind = surface->kind;
    if (kind != CPM_SURF_CIRCLE && kind != CPM_SURF_SPHERE && kind != CPM_SURF_TORUS)
      CPM_FAIL(CPM_E_INVALID, "unknown surface kind %d", kind);
    if (!(surface->R > 0) || (kind == CPM_SURF_TORUS && !(surface->rho > 0 && surface->rho < surface->R)))
      CPM_FAIL(CPM_E_INVALID, "bad surface radii");
    for (int c = 0; c < n_ibc; ++c) {
      const int k = ibcs[c].kind;
      const bool arc_ok = k != CPM_IBC_LATITUDE_ARC ||
                          (std::hypot(ibcs[c].arc[0], ibcs[c].arc[1]) > 0.5 &&
                           std::hypot(ibcs[c].arc[2], ibcs[c].arc[3]) > 0.5);
      const bool ok = k == CPM_IBC_POINT ||
                      ((k == CPM_IBC_LATITUDE || k == CPM_IBC_LATITUDE_ARC) &&
                       kind == CPM_SURF_SPHERE && std::fabs(ibcs[c].z0) < surface->R && arc_ok) ||
                      (k == CPM_IBC_MERIDIAN && kind == CPM_SURF_TORUS);
      if (!ok) CPM_FAIL(CPM_E_INVALID, "interior boundary %d (kind %d) does not fit surface kind %d", c, k, kind);
      for (int s2 = 0; s2 < 2; ++s2) {
        const int bc = ibcs[c].bc[s2];
        if (bc != CPM_BC_DIRICHLET && bc != CPM_BC_NEUMANN)
          CPM_FAIL(CPM_E_INVALID, "interior boundary %d: unknown condition %d", c, bc);
        // a conormal direction does not exist at a point C of a surface; a
        // point of a curve in R^2 has one (the curve's own direction)
        if (bc == CPM_BC_NEUMANN && k == CPM_IBC_POINT && kind != CPM_SURF_CIRCLE)
          CPM_FAIL(CPM_E_INVALID, "interior boundary %d: a zero-Neumann condition is not "
                   "defined at a point of a surface", c);
      }
    }
    hipStream_t st = (hipStream_t)hip_stream;
    std::unique_ptr<cpm_band> b(new cpm_band());
    if (allocator) b->da.a = *allocator;
    b->da.st = st;
    CPM_HIP(hipGetDevice(&b->device));
    b->dim = kind == CPM_SURF_CIRCLE ? 2 : 3;
    b->N = grid->N;
    b->order = grid->order;
    b->p = grid->p;
    b->surf = *surface;
    if (b->dim == 2) b->surf.center[2] = 0.0;
    b->n_ibc = n_ibc;
    b->ibcs.assign(ibcs, ibcs + n_ibc);
    b->h = 1.0 / grid->N;
    // eq. (bandwidth), q = 1: (d - 1) ((p + 1) / 2)^2 + (1 + (p + 1) / 2)^2, i.e.
    // 17 / 13 (cubic, R^3 / R^2) and 10.75 / 8.5 (quadratic)
    const double hp = 0.5 * (double)(grid->p + 1);
    const double K = (double)(b->dim - 1) * (hp * hp) + (1.0 + hp) * (1.0 + hp);
    b->r = grid->r_band > 0 ? grid->r_band : std::sqrt(K) / (double)grid->N;
    b->tau = (grid->tau_factor > 0 ? grid->tau_factor : 0.1) / (double)((int64_t)grid->N * grid->N);
    b->check_factor = grid->check_factor > 0 ? grid->check_factor : 2.0;
    if (grid->check_reach && !(b->r < reach_of(*surface)))
      CPM_FAIL(CPM_E_REACH, "band radius %.6g is not below the reach %.6g of the surface "
               "(h must be smaller)", b->r, reach_of(*surface));
    if (grid->band != CPM_BAND_TUBE && grid->band != CPM_BAND_STENCIL_SET)
      CPM_FAIL(CPM_E_INVALID, "unknown band kind %d", grid->band);
    if (grid->band == CPM_BAND_STENCIL_SET) {
      // the tube first, then the same construction restricted to its
      // stencil set (a node filter in the classification pass)
      std::unique_ptr<cpm_band> t(new cpm_band());
      t->da = b->da;
      t->device = b->device;
      t->dim = b->dim;
      t->N = b->N;
      t->order = b->order;
      t->p = b->p;
      t->surf = b->surf;
      t->n_ibc = b->n_ibc;
      t->ibcs = b->ibcs;
      t->h = b->h;
      t->r = b->r;
      t->tau = b->tau;
      t->check_factor = b->check_factor;
      if (b->dim == 3) build<3>(t.get(), st, Filter{});
      else build<2>(t.get(), st, Filter{});
      Tmp<unsigned long long> keep(b.get(), t->nb);
      const Filter F = b->dim == 3 ? stencil_set_filter<3>(t.get(), st, keep.p)
                                   : stencil_set_filter<2>(t.get(), st, keep.p);
      if (b->dim == 3) build<3>(b.get(), st, F);
      else build<2>(b.get(), st, F);
      CPM_HIP(hipStreamSynchronize(st));
      b->band_kind = CPM_BAND_STENCIL_SET;
    } else {
      if (b->dim == 3) build<3>(b.get(), st, Filter{});
      else build<2>(b.get(), st, Filter{});
    }
    *out = b.release();
  });
}

extern "C" cpm_status cpm_band_export(const cpm_band* b, int what, void* host_dst, size_t bytes) {
  return guard([&] {
    if (!b || !host_dst) CPM_FAIL(CPM_E_INVALID, "null argument");
    const int d = b->dim, nm = d == 3 ? 64 : 16;
    size_t need = 0;
    switch (what) {
      case CPM_EXPORT_COORDS: need = (size_t)b->n_s * d * 4; break;
      case CPM_EXPORT_CP: need = (size_t)b->n_s * d * 8; break;
      case CPM_EXPORT_BC_NODE: case CPM_EXPORT_BC_SIDE: case CPM_EXPORT_BC_CURVE:
        need = (size_t)b->n_c * 4; break;
      case CPM_EXPORT_BC_CPC: need = (size_t)b->n_c * d * 8; break;
      case CPM_EXPORT_ECOLS: need = (size_t)b->n * nm * 4; break;
      case CPM_EXPORT_LCOLS: need = (size_t)b->n * 2 * d * 4; break;
      case CPM_EXPORT_BASE: need = (size_t)b->n * d * 4; break;
      default: CPM_FAIL(CPM_E_INVALID, "unknown export item %d", what);
    }
    if (bytes != need) CPM_FAIL(CPM_E_INVALID, "export %d needs %zu bytes, got %zu", what, need, bytes);
    if (need == 0) return;
    hipStream_t st = nullptr;
    if (what == CPM_EXPORT_CP) {
      std::vector<double> soa((size_t)b->n_s * d);
      CPM_HIP(hipMemcpy(soa.data(), b->cp, soa.size() * 8, hipMemcpyDeviceToHost));
      double* o = static_cast<double*>(host_dst);
      for (int64_t i = 0; i < b->n_s; ++i)
        for (int a = 0; a < d; ++a) o[i * d + a] = soa[(size_t)a * b->n_s + i];
      return;
    }
    const void* src = nullptr;
    if (what == CPM_EXPORT_BC_NODE) src = b->bc_node;
    if (what == CPM_EXPORT_BC_SIDE) src = b->bc_side;
    if (what == CPM_EXPORT_BC_CURVE) src = b->bc_curve;
    if (what == CPM_EXPORT_BC_CPC) src = b->bc_cpc;
    if (src) {
      CPM_HIP(hipMemcpy(host_dst, src, need, hipMemcpyDeviceToHost));
      return;
    }
    Tmp<int> dev(b, need / 4);
    CPM_HIP(hipMemset(dev.p, 0xff, need));
    int* coords = what == CPM_EXPORT_COORDS ? dev.p : nullptr;
    int* ecols = what == CPM_EXPORT_ECOLS ? dev.p : nullptr;
    int* lcols = what == CPM_EXPORT_LCOLS ? dev.p : nullptr;
    int* bases = what == CPM_EXPORT_BASE ? dev.p : nullptr;
    if (bases) CPM_HIP(hipMemset(dev.p, 0, need));
    if (d == 3) export_rows<3>(b, coords, ecols, lcols, bases, st);
    else export_rows<2>(b, coords, ecols, lcols, bases, st);
    CPM_HIP(hipStreamSynchronize(st));
    CPM_HIP(hipMemcpy(host_dst, dev.p, need, hipMemcpyDeviceToHost));
  });
}
