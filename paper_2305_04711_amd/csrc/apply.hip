// The CPM operator A = m I + n [diag L + (L - diag L) E] (Sec. 5.4) and its
// transpose, matrix-free, in two passes (the paper's four steps with steps 3
// and 4 folded into the second pass):
//   pass 1  a = E u          (eq. interp-stencil)  k_gather + k_gather_rows
//   pass 2  v = (m + n D) u + n N^2 sum_nbr a      k_lap    + k_lap_rows
// Pass 1 runs one workgroup per gather tile: the rows whose stencil base lies
// in one block.  Their 4^d members lie in the 2^d blocks starting at that
// block, which the workgroup stages in LDS as a dense (2 BX)^d cube before
// every row reads its members from LDS.  Rows whose stencils were changed by
// an interior boundary (and every BC row) are explicit rows with stored
// columns and weights.  Pass 2 maps one wavefront to one block of 64 nodes
// and finds face neighbours through the block neighbour table; rows with
// swapped FD neighbours (and BC rows) are explicit.
#include <mutex>

#include "cpm_internal.hpp"
#include "lagrange.hpp"

namespace cpm {

struct BlockView {
  const unsigned long long* mask;
  const int* off;
  const int* nbr;
  const unsigned long long* lrow_mask;
  const QMeta* face;
  int nb;
};

static BlockView bview(const cpm_band* b) {
  return BlockView{b->blk_mask, b->blk_off, b->blk_nbr, b->lrow_mask, b->blk_face, b->nb};
}

// Wave-uniform broadcast of lane k (k must be the same in every lane).
__device__ __forceinline__ int lane_i32(int v, int k) { return __builtin_amdgcn_readlane(v, k); }
__device__ __forceinline__ unsigned long long lane_u64(unsigned long long v, int k) {
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)v, k);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(v >> 32), k);
  return ((unsigned long long)hi << 32) | lo;
}

// With a wave-uniform mask m (in scalar registers): base + the number of
// bits of m below the lane (masked bit counts, two vector instructions), and
// whether the lane's own bit is set (the mask used as an execution mask).
__device__ __forceinline__ int lane_count_below(unsigned long long m, int base) {
  return (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                        __builtin_amdgcn_mbcnt_lo((unsigned)m, (unsigned)base));
}
__device__ __forceinline__ bool lane_in(unsigned long long m) {
  return __builtin_amdgcn_inverse_ballot_w64(m);
}

// Workgroups are dispatched to the 8 XCDs round robin; this bijection on
// [0, g) gives each XCD a contiguous range of work items so that neighbouring
// tiles, which stage the same blocks, share one L2.
__device__ __forceinline__ int xcd_remap(int b, int g) {
  const int q = g >> 3, r = g & 7, x = b & 7, k = b >> 3;
  return x * q + (x < r ? x : r) + k;
}

struct TileView {
  const int* tile_inst;   // batched composite: instance of each tile (else null)
  const int* skip;        // batched composite: instances to skip (else null)
  const QMeta* meta;
  const int* tile_blk;
  const int* tile_start;
  const int* perm;
  const double* frac64;
  const float* frac32;
  const unsigned* lbase;
  int ntr;
  int p;                  // interpolation degree: 3, or 2 (fourth weight 0)
};

static TileView tview(const cpm_band* b) {
  return TileView{b->tile_inst, b->inst_skip, b->tile_meta, b->tile_blk, b->tile_start, b->perm,
                  b->frac64, b->frac32, b->lbase, b->n_tile_rows, b->p};
}

template <int DIM> struct Cube {
  static constexpr int E = 2 * Geo<DIM>::BX;              // cube edge
  static constexpr int SIZE = DIM == 3 ? E * E * E : E * E;
};

// Per-row stencil base (local to the tile block) and fraction.  The fraction
// is stored in the vector precision TS (FP64 or FP32) and returned in FP64:
// the weights are always evaluated in FP64, so they sum to one to FP64
// rounding whatever precision the fraction was stored in.
template <class TS>
__device__ __forceinline__ const TS* frac_of(const TileView& tv);
template <>
__device__ __forceinline__ const double* frac_of<double>(const TileView& tv) { return tv.frac64; }
template <>
__device__ __forceinline__ const float* frac_of<float>(const TileView& tv) { return tv.frac32; }

template <class TS, int DIM>
__device__ __forceinline__ void row_stencil(const TileView& tv, int pos, int lb[3], double t[3]) {
  const unsigned p = tv.lbase[pos];
  const TS* fr = frac_of<TS>(tv);
  lb[0] = p & 0xff;
  lb[1] = (p >> 8) & 0xff;
  lb[2] = DIM == 3 ? (p >> 16) & 0xff : 0;
#pragma unroll
  for (int a = 0; a < DIM; ++a) t[a] = (double)fr[(int64_t)a * tv.ntr + pos];
  if (DIM == 2) t[2] = 0.0;
}

// ---------------------------------------------------------------- pass 1
// Interpolation of one row from the staged cube (sum-factorised tensor
// product): x lines first, then y, then z.  FP64 arithmetic.
// NP = p + 1 stencil nodes per axis (4 cubic, 3 quadratic).
template <int DIM, int NR, int CSZ, int E, int EP, class TL, int NP>
__device__ __forceinline__ void interp_row_np(const TL (&s_u)[NR][CSZ], const double wx[4],
                                              const double wy[4], const double wz[4],
                                              const int lb[3], double acc[NR]) {
  const int lx = lb[0], ly = lb[1], lz = lb[2];
#pragma unroll
  for (int r = 0; r < NR; ++r) acc[r] = 0.0;
  if (DIM == 3) {
#pragma unroll
    for (int c = 0; c < NP; ++c) {
      double accz[NR];
#pragma unroll
      for (int r = 0; r < NR; ++r) accz[r] = 0.0;
#pragma unroll
      for (int b = 0; b < NP; ++b) {
        const int base = ((lz + c) * E + (ly + b)) * EP + lx;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          const TL* row = &s_u[r][base];
          double x = wx[0] * (double)row[0] + wx[1] * (double)row[1] + wx[2] * (double)row[2];
          if (NP == 4) x += wx[3] * (double)row[3];
          accz[r] += wy[b] * x;
        }
      }
#pragma unroll
      for (int r = 0; r < NR; ++r) acc[r] += wz[c] * accz[r];
    }
  } else {
#pragma unroll
    for (int b = 0; b < NP; ++b) {
      const int base = (ly + b) * EP + lx;
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const TL* row = &s_u[r][base];
        double x = wx[0] * (double)row[0] + wx[1] * (double)row[1] + wx[2] * (double)row[2];
        if (NP == 4) x += wx[3] * (double)row[3];
        acc[r] += wy[b] * x;
      }
    }
  }
}

// NP = 4 serves cubic rows and quadratic rows in the padded layout (fourth
// weight 0); NP = 3 is the quadratic form of the non-persistent tile gather:
// 27 members and 39 multiply-adds instead of 64 and 84 (both forms give the
// same sums up to the sign of a zero).
template <int DIM, int NR, int CSZ, int E, int EP, class TL, int NP = 4>
__device__ __forceinline__ void interp_row(const TL (&s_u)[NR][CSZ], int p, const int lb[3],
                                           const double tt[3], double acc[NR]) {
  double wx[4], wy[4], wz[4] = {0.0, 0.0, 0.0, 0.0};
  lagrange_p<double>(NP == 3 ? 2 : p, tt[0], wx);
  lagrange_p<double>(NP == 3 ? 2 : p, tt[1], wy);
  if (DIM == 3) lagrange_p<double>(NP == 3 ? 2 : p, tt[2], wz);
  interp_row_np<DIM, NR, CSZ, E, EP, TL, NP>(s_u, wx, wy, wz, lb, acc);
}

// One wavefront per tile: stage the (2 BX)^d cube of u into LDS (x lines
// padded by PAD elements to spread LDS banks), then each lane interpolates
// rows of the tile.  The staged blocks' masks and first DOFs are
// wave-uniform: scalar loads, and a staged node's DOF and presence come from
// masked bit counts and an execution mask instead of per-lane 64-bit mask
// arithmetic (the kernel is limited by instruction issue as much as by
// memory).  u is stored and staged in TS (FP64 or FP32: an FP32 value is
// staged exactly); weights, products and sums are FP64 and
// a is written in FP64 for both storage precisions: the Laplacian pass differences neighbouring
// values of a and scales the difference by N^2, so a rounding of a to FP32
// would be amplified by N^2 (on the smooth modes that converge last, a
// relative error of order eps32 ||A|| / lambda_min in A u).
// At most 6 waves per SIMD keeps the register use in check (left to itself
// the compiler hoists every LDS read of a row and the occupancy drops to 4
// waves per SIMD, about 1.5x slower).
template <class TS, int DIM, int NR, int PAD, int NP = 4>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(6))) void k_gather(
    BlockView B, TileView tv, int N, const TS* __restrict__ u, double* __restrict__ a, int64_t ld,
    int xcd) {
  using G = Geo<DIM>;
  constexpr int E = Cube<DIM>::E, EP = E + PAD, NQ = 1 << DIM;
  constexpr int CS = DIM == 3 ? E * E * EP : E * EP;
  __shared__ TS s_u[NR][CS];
  const int t = xcd ? xcd_remap(blockIdx.x, gridDim.x) : blockIdx.x;
  const int lane = threadIdx.x;
  if (tv.skip && tv.skip[tv.tile_inst[t]]) return;   // converged batch instance
  // the staged blocks' masks and first DOFs: wave-uniform, scalar loads
  const QMeta* tm = tv.meta + (int64_t)t * 8;
  const int cx0 = G::lx(lane), cy0 = G::ly(lane), cz0 = G::lz(lane);
  // the first pass's row data is requested before the staging loads, and
  // every pass requests the next pass's before interpolating
  const int beg = tv.tile_start[t], end = tv.tile_start[t + 1];
  int lb[3] = {0, 0, 0};
  double tt[3] = {0.0, 0.0, 0.0};
  if (beg + lane < end) row_stencil<TS, DIM>(tv, beg + lane, lb, tt);
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const unsigned long long m = tm[q].mask;
    const int qx = q & 1, qy = (q >> 1) & 1, qz = DIM == 3 ? (q >> 2) : 0;
    const int cx = qx * G::BX + cx0, cy = qy * G::BX + cy0, cz = qz * G::BX + cz0;
    const int ci = DIM == 3 ? (cz * E + cy) * EP + cx : cy * EP + cx;
    const int dof = lane_count_below(m, tm[q].off);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      TS x = TS(0);
      if (lane_in(m)) x = u[r * ld + dof];
      s_u[r][ci] = x;
    }
  }
  __syncthreads();
  for (int pos = beg + lane; pos < end; pos += 64) {
    const int lbc[3] = {lb[0], lb[1], lb[2]};
    const double tc[3] = {tt[0], tt[1], tt[2]};
    const int dof = tv.perm[pos];
    if (pos + 64 < end) row_stencil<TS, DIM>(tv, pos + 64, lb, tt);
    double acc[NR];
    interp_row<DIM, NR, CS, E, EP, TS, NP>(s_u, tv.p, lbc, tc, acc);
#pragma unroll
    for (int r = 0; r < NR; ++r) a[r * ld + dof] = acc[r];
  }
}

// Persistent form of k_gather: XCD x (workgroup id mod 8) owns a contiguous
// eighth of the tiles, and its W waves take every W-th tile of that range.
// While a tile's blocks are staged, the wave already requests the next
// tile's metadata and row range, so a tile costs one dependent round trip to
// memory instead of two.
template <class TS, int DIM, int NR, int PAD>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(6))) void k_gather_ps(
    BlockView B, TileView tv, int N, const TS* __restrict__ u, double* __restrict__ a, int64_t ld,
    int ntiles) {
  using G = Geo<DIM>;
  constexpr int E = Cube<DIM>::E, EP = E + PAD, NQ = 1 << DIM;
  constexpr int CS = DIM == 3 ? E * E * EP : E * EP;
  __shared__ TS s_u[NR][CS];
  const int lane = threadIdx.x;
  const int x = blockIdx.x & 7, wk = blockIdx.x >> 3, W = gridDim.x >> 3;
  const int q8 = ntiles >> 3, r8 = ntiles & 7;
  const int lo = x * q8 + (x < r8 ? x : r8), hi = lo + q8 + (x < r8 ? 1 : 0);
  int t = lo + wk;
  if (t >= hi) return;
  unsigned long long qm = 0ull;
  int qoff = 0;
  if (lane < NQ) {
    const QMeta q = tv.meta[(int64_t)t * 8 + lane];
    qm = q.mask;
    qoff = q.off;
  }
  int beg = tv.tile_start[t], end = tv.tile_start[t + 1];
  const int cx0 = G::lx(lane), cy0 = G::ly(lane), cz0 = G::lz(lane);
  while (true) {
    const int tn = t + W;
    const bool more = tn < hi;
    int lb[3] = {0, 0, 0};
    double tt[3] = {0.0, 0.0, 0.0};
    if (beg + lane < end) row_stencil<TS, DIM>(tv, beg + lane, lb, tt);
    TS sv[NQ][NR];
    int sci[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const unsigned long long m = lane_u64(qm, q);
      const int off = lane_i32(qoff, q);
      const int qx = q & 1, qy = (q >> 1) & 1, qz = DIM == 3 ? (q >> 2) : 0;
      const int cx = qx * G::BX + cx0, cy = qy * G::BX + cy0, cz = qz * G::BX + cz0;
      sci[q] = DIM == 3 ? (cz * E + cy) * EP + cx : cy * EP + cx;
      const bool on = (m >> lane) & 1ull;
      const int dof = off + __popcll(m & ((1ull << lane) - 1ull));
#pragma unroll
      for (int r = 0; r < NR; ++r) sv[q][r] = on ? u[r * ld + dof] : TS(0);
    }
    unsigned long long qm_n = 0ull;
    int qoff_n = 0, beg_n = 0, end_n = 0;
    if (more) {
      if (lane < NQ) {
        const QMeta q = tv.meta[(int64_t)tn * 8 + lane];
        qm_n = q.mask;
        qoff_n = q.off;
      }
      beg_n = tv.tile_start[tn];
      end_n = tv.tile_start[tn + 1];
    }
    __syncthreads();   // the previous tile's rows are done with the cube
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
      for (int r = 0; r < NR; ++r) s_u[r][sci[q]] = sv[q][r];
    __syncthreads();
    for (int pos = beg + lane; pos < end; pos += 64) {
      const int lbc[3] = {lb[0], lb[1], lb[2]};
      const double tc[3] = {tt[0], tt[1], tt[2]};
      const int dof = tv.perm[pos];
      if (pos + 64 < end) row_stencil<TS, DIM>(tv, pos + 64, lb, tt);
      double acc[NR];
      interp_row<DIM, NR, CS, E, EP, TS>(s_u, tv.p, lbc, tc, acc);
#pragma unroll
      for (int r = 0; r < NR; ++r) a[r * ld + dof] = acc[r];
    }
    if (!more) break;
    t = tn;
    qm = qm_n;
    qoff = qoff_n;
    beg = beg_n;
    end = end_n;
  }
}

// Persistent and pipelined form: as k_gather_ps, but the staging loads of a
// wave's next tile (with that tile's first row data and the metadata of the
// one after) are issued as soon as the current tile's cube is in LDS and its
// first two passes of row data are requested, so they are in flight while
// the current tile's rows are interpolated.  (Vector memory requests of a
// wave complete in issue order, so everything the current tile waits for is
// requested before the next tile's staging.)  A wave holds one tile's staged
// values in registers at a time.
template <class TS, int DIM, int NR, int PAD>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(5))) void k_gather_pp(
    BlockView B, TileView tv, int N, const TS* __restrict__ u, double* __restrict__ a, int64_t ld,
    int ntiles) {
  using G = Geo<DIM>;
  constexpr int E = Cube<DIM>::E, EP = E + PAD, NQ = 1 << DIM;
  constexpr int CS = DIM == 3 ? E * E * EP : E * EP;
  __shared__ TS s_u[NR][CS];
  const int lane = threadIdx.x;
  const int x = blockIdx.x & 7, wk = blockIdx.x >> 3, W = gridDim.x >> 3;
  const int q8 = ntiles >> 3, r8 = ntiles & 7;
  const int lo = x * q8 + (x < r8 ? x : r8), hi = lo + q8 + (x < r8 ? 1 : 0);
  int t = lo + wk;
  if (t >= hi) return;
  const int cx0 = G::lx(lane), cy0 = G::ly(lane), cz0 = G::lz(lane);
  int sci[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int qx = q & 1, qy = (q >> 1) & 1, qz = DIM == 3 ? (q >> 2) : 0;
    const int cx = qx * G::BX + cx0, cy = qy * G::BX + cy0, cz = qz * G::BX + cz0;
    sci[q] = DIM == 3 ? (cz * E + cy) * EP + cx : cy * EP + cx;
  }
  // staging values, first-pass row data and row range of tile tt
  auto stage = [&](int tt, unsigned long long qm, int qoff, TS (&sv)[NQ][NR], int lb[3],
                   double t3[3], int& dof, int& beg, int& end) {
    beg = tv.tile_start[tt];
    end = tv.tile_start[tt + 1];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const unsigned long long m = lane_u64(qm, q);
      const int off = lane_i32(qoff, q);
      const bool on = (m >> lane) & 1ull;
      const int d = off + __popcll(m & ((1ull << lane) - 1ull));
#pragma unroll
      for (int r = 0; r < NR; ++r) sv[q][r] = on ? u[r * ld + d] : TS(0);
    }
    lb[0] = lb[1] = lb[2] = 0;
    t3[0] = t3[1] = t3[2] = 0.0;
    dof = -1;
    if (beg + lane < end) {
      row_stencil<TS, DIM>(tv, beg + lane, lb, t3);
      dof = tv.perm[beg + lane];
    }
  };
  auto meta = [&](int tt, unsigned long long& qm, int& qoff) {
    qm = 0ull;
    qoff = 0;
    if (tt < hi && lane < NQ) {
      const QMeta q = tv.meta[(int64_t)tt * 8 + lane];
      qm = q.mask;
      qoff = q.off;
    }
  };
  auto rows = [&](const int lbr[3], const double tr[3], int dof) {
    double acc[NR];
    interp_row<DIM, NR, CS, E, EP, TS>(s_u, tv.p, lbr, tr, acc);
    if (dof >= 0) {
#pragma unroll
      for (int r = 0; r < NR; ++r) a[r * ld + dof] = acc[r];
    }
  };
  unsigned long long qm;
  int qoff;
  meta(t, qm, qoff);
  TS sv[NQ][NR];
  int lb[3], dof, beg, end;
  double t3[3];
  stage(t, qm, qoff, sv, lb, t3, dof, beg, end);
  meta(t + W, qm, qoff);
  while (true) {
    __syncthreads();   // the previous tile's rows are done with the cube
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
      for (int r = 0; r < NR; ++r) s_u[r][sci[q]] = sv[q][r];
    __syncthreads();
    const int lb1[3] = {lb[0], lb[1], lb[2]};
    const double t1[3] = {t3[0], t3[1], t3[2]};
    const int dof1 = dof, cbeg = beg, cend = end;
    // the second pass's row data before the next tile's staging
    int lb2[3] = {0, 0, 0}, dof2 = -1;
    double t2[3] = {0.0, 0.0, 0.0};
    if (cbeg + 64 + lane < cend) {
      row_stencil<TS, DIM>(tv, cbeg + 64 + lane, lb2, t2);
      dof2 = tv.perm[cbeg + 64 + lane];
    }
    const int tn = t + W;
    const bool more = tn < hi;
    if (more) {
      stage(tn, qm, qoff, sv, lb, t3, dof, beg, end);
      meta(tn + W, qm, qoff);
    }
    if (cbeg < cend) rows(lb1, t1, dof1);
    if (cbeg + 64 < cend) rows(lb2, t2, dof2);
    for (int pos = cbeg + 128 + lane; pos - lane < cend; pos += 64) {
      int lbr[3] = {0, 0, 0}, dr = -1;
      double tr[3] = {0.0, 0.0, 0.0};
      if (pos < cend) {
        row_stencil<TS, DIM>(tv, pos, lbr, tr);
        dr = tv.perm[pos];
      }
      rows(lbr, tr, dr);
    }
    if (!more) break;
    t = tn;
  }
}

template <class T>
__device__ __forceinline__ T wave_sum(T v, int width) {
  for (int o = width >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, width);
  return v;
}

// Wavefront sums of d0 and d1 (every lane of the wave must call it), written
// by lane 0 to part[idx] and part[np + idx] with idx = first + the wave's
// index in its workgroup: the partials of a fused dot product, one per
// wavefront, finished in a fixed order by the solver.
__device__ __forceinline__ void wave_dot2(double d0, double d1, double* part, int np, int first) {
  d0 = wave_sum(d0, 64);
  d1 = wave_sum(d1, 64);
  if ((threadIdx.x & 63) == 0) {
    const int idx = first + (threadIdx.x >> 6);
    part[idx] = d0;
    part[np + idx] = d1;
  }
}

// Explicit interpolation rows: a[id] = sum_o w_o u[col_o]; nm lanes per row
// (nm = 4^d: a wavefront in 3-D, a quarter wavefront in 2-D), lane = member.
// FP64 weights for both storage precisions (the interior-boundary rows keep
// their FP64 closest-point weights), FP64 sums into the FP64 a.
template <class TS>
__global__ __launch_bounds__(256) void k_gather_rows(int nrows, int nm, const int* __restrict__ row_id,
                                                     const int* __restrict__ col,
                                                     const double* __restrict__ w,
                                                     const TS* __restrict__ u,
                                                     double* __restrict__ a, int64_t ld, int nrhs,
                                                     const int* __restrict__ row_inst,
                                                     const int* __restrict__ skip) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = g / nm;
  const int o = (int)(g % nm);
  const bool live = i < nrows && !(skip && skip[row_inst[i]]);
  const int c = live ? col[i * nm + o] : -1;
  const double wt = live ? w[i * nm + o] : 0.0;
  for (int r = 0; r < nrhs; ++r) {
    double v = c >= 0 ? wt * (double)u[r * ld + c] : 0.0;
    v = wave_sum(v, nm);
    if (live && o == 0) a[r * ld + row_id[i]] = v;
  }
}

// ---------------------------------------------------------------- pass 2
// cd u + co s with one explicit rounding order, shared by both forms of the
// pass so that they agree bit for bit whatever the compiler contracts.
__device__ __forceinline__ double lap_out(double cd, double u, double co, double s) {
  return __fma_rn(co, s, cd * u);
}

// v = cd u + co sum_nbr a (+ gauge); lane = slot; each wavefront handles KB
// consecutive blocks so that their loads are in flight together.  Lanes
// 8j..8j+7 load block j's metadata (its own and its face neighbours' masks
// and first DOFs, and the explicit-row mask), broadcast with readlane, so each
// lane finds its neighbours' DOFs by arithmetic.  ALL = false skips rows with
// explicit FD stencils and reads u for the diagonal term; ALL = true
// (transpose) visits every PDE row and writes co sum_nbr a only.  TU, TA, TV
// are the storage types of u, a and v; the arithmetic is FP64.
constexpr int kLapBlocksPerWave = 2;

template <class TU, class TA, class TV, int DIM, bool ALL, bool DOT = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void k_lap(
    BlockView B, const TU* __restrict__ u, const TA* __restrict__ a, TV* __restrict__ v,
    int64_t ld, int nrhs, double cd, double co, const double* __restrict__ gsum, double gscale,
    int xcd, const double* __restrict__ coef, const int* __restrict__ skip,
    const TV* __restrict__ dy = nullptr, double* __restrict__ dpart = nullptr, int dnp = 0) {
  using G = Geo<DIM>;
  constexpr int KB = kLapBlocksPerWave;
  const int wg = xcd ? xcd_remap(blockIdx.x, gridDim.x) : blockIdx.x;
  const int blk0 = (wg * 4 + (threadIdx.x >> 6)) * KB;
  const int slot = threadIdx.x & 63;
  // with DOT every wave takes part in the workgroup's reduction
  if (!DOT && blk0 >= B.nb) return;
  unsigned long long lm = 0ull;
  int loff = 0, lpad = 0;
  {
    const int j = slot >> 3, e = slot & 7;
    if (j < KB && blk0 + j < B.nb) {
      const QMeta q = B.face[(int64_t)(blk0 + j) * 8 + e];
      lm = q.mask;
      loff = q.off;
      lpad = q.pad;
    }
  }
  // batched systems: per-instance (cd, co), instance id in entry 7's pad
  double cdj[KB], coj[KB];
  bool skipj[KB];
#pragma unroll
  for (int j = 0; j < KB; ++j) {
    cdj[j] = cd;
    coj[j] = co;
    skipj[j] = false;
    if (coef) {
      const int inst = lane_i32(lpad, 8 * j + 7);
      const int ii = inst > 0 ? inst : 0;
      cdj[j] = coef[2 * ii];
      coj[j] = coef[2 * ii + 1];
      skipj[j] = skip && skip[ii];
    }
  }
  const int l[3] = {G::lx(slot), G::ly(slot), G::lz(slot)};
  int dof[KB];
  int nd[KB][2 * DIM];
#pragma unroll
  for (int j = 0; j < KB; ++j) {
    const unsigned long long m = lane_u64(lm, 8 * j);
    const int off0 = lane_i32(loff, 8 * j);
    const unsigned long long xm = lane_u64(lm, 8 * j + 7);
    bool on = ((m >> slot) & 1ull) && !skipj[j];
    if (!ALL && ((xm >> slot) & 1ull)) on = false;
    dof[j] = on ? off0 + __popcll(m & ((1ull << slot) - 1ull)) : -1;
#pragma unroll
    for (int f = 0; f < 2 * DIM; ++f) {
      const unsigned long long fmk = lane_u64(lm, 8 * j + f + 1);
      const int fof = lane_i32(loff, 8 * j + f + 1);
      int q[3] = {l[0], l[1], l[2]};
      q[f >> 1] += (f & 1) ? 1 : -1;
      const bool out = q[f >> 1] < 0 || q[f >> 1] >= G::BX;
      q[f >> 1] &= G::BX - 1;
      const int s2 = G::slot(q[0], q[1], q[2]);
      const unsigned long long mm = out ? fmk : m;
      const int oo = out ? fof : off0;
      nd[j][f] = ((mm >> s2) & 1ull) ? oo + __popcll(mm & ((1ull << s2) - 1ull)) : -1;
    }
  }
  if constexpr (DOT) {
    // the solver's fused dot products: one right-hand side; y is requested
    // together with u so that it adds no round trip to memory
    double uv[KB], yv[KB], s[KB];
#pragma unroll
    for (int j = 0; j < KB; ++j) {
      uv[j] = dof[j] >= 0 ? (double)u[dof[j]] : 0.0;
      yv[j] = dof[j] >= 0 ? (double)dy[dof[j]] : 0.0;
      s[j] = 0.0;
#pragma unroll
      for (int f = 0; f < 2 * DIM; ++f)
        if (dof[j] >= 0 && nd[j][f] >= 0) s[j] += (double)a[nd[j][f]];
    }
    double d0 = 0.0, d1 = 0.0;
#pragma unroll
    for (int j = 0; j < KB; ++j) {
      if (dof[j] < 0) continue;
      double o = lap_out(cdj[j], uv[j], coj[j], s[j]);
      if (gsum) o += gscale * gsum[0];
      const TV ov = (TV)o;
      v[dof[j]] = ov;
      d0 += yv[j] * (double)ov;
      d1 += (double)ov * (double)ov;
    }
    wave_dot2(d0, d1, dpart, dnp, blockIdx.x * 4);
    return;
  }
  for (int r = 0; r < nrhs; ++r) {
    double out[KB];
#pragma unroll
    for (int j = 0; j < KB; ++j) {
      double s = 0.0;
#pragma unroll
      for (int f = 0; f < 2 * DIM; ++f)
        if (dof[j] >= 0 && nd[j][f] >= 0) s += (double)a[r * ld + nd[j][f]];
      if constexpr (ALL) out[j] = coj[j] * s;
      else out[j] = dof[j] >= 0 ? lap_out(cdj[j], (double)u[r * ld + dof[j]], coj[j], s) : 0.0;
    }
#pragma unroll
    for (int j = 0; j < KB; ++j) {
      if (dof[j] < 0) continue;
      double o = out[j];
      if (gsum) o += gscale * gsum[r];
      v[r * ld + dof[j]] = (TV)o;
    }
  }
}

// The same pass with neighbour values exchanged between lanes: each lane
// loads u and a of its own slot (one coalesced load each: a block's DOFs are
// contiguous), takes the values of in-block face neighbours from the lanes
// holding them (cross-lane moves; an absent slot holds 0, which drops that
// neighbour as the pass requires), and only the lanes on a block face load
// the neighbour across it.  Fewer and narrower memory requests per block
// than k_lap, which gathers every neighbour from memory.
template <class T>
__device__ __forceinline__ T lane_take(T v, int src) {
  if constexpr (sizeof(T) == 8) {
    const long long b = __double_as_longlong((double)v);
    const int lo = __shfl((int)(unsigned)(b & 0xffffffffll), src, 64);
    const int hi = __shfl((int)(b >> 32), src, 64);
    return (T)__longlong_as_double(((long long)hi << 32) | (unsigned)lo);
  } else {
    return __shfl(v, src, 64);
  }
}

constexpr int kLapShBlocksPerWave = 1;

template <class TU, class TA, class TV, int DIM, bool ALL, bool DOT = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void k_lap_sh(
    BlockView B, const TU* __restrict__ u, const TA* __restrict__ a, TV* __restrict__ v,
    int64_t ld, int nrhs, double cd, double co, const double* __restrict__ gsum, double gscale,
    int xcd, const double* __restrict__ coef, const int* __restrict__ skip,
    const TV* __restrict__ dy = nullptr, double* __restrict__ dpart = nullptr, int dnp = 0) {
  using G = Geo<DIM>;
  constexpr int KB = kLapShBlocksPerWave;
  const int wg = xcd ? xcd_remap(blockIdx.x, gridDim.x) : blockIdx.x;
  const int blk0 = (wg * 4 + (threadIdx.x >> 6)) * KB;
  const int slot = threadIdx.x & 63;
  if (!DOT && blk0 >= B.nb) return;
  unsigned long long lm = 0ull;
  int loff = 0, lpad = 0;
  {
    const int j = slot >> 3, e = slot & 7;
    if (j < KB && blk0 + j < B.nb) {
      const QMeta q = B.face[(int64_t)(blk0 + j) * 8 + e];
      lm = q.mask;
      loff = q.off;
      lpad = q.pad;
    }
  }
  const int l[3] = {G::lx(slot), G::ly(slot), G::lz(slot)};
  double cdj[KB], coj[KB];
  int own[KB], outr[KB], nsrc[KB][2 * DIM];
#pragma unroll
  for (int j = 0; j < KB; ++j) {
    cdj[j] = cd;
    coj[j] = co;
    bool skipj = false;
    if (coef) {
      const int inst = lane_i32(lpad, 8 * j + 7);
      const int ii = inst > 0 ? inst : 0;
      cdj[j] = coef[2 * ii];
      coj[j] = coef[2 * ii + 1];
      skipj = skip && skip[ii];
    }
    const unsigned long long m = lane_u64(lm, 8 * j);
    const int off0 = lane_i32(loff, 8 * j);
    const unsigned long long xm = lane_u64(lm, 8 * j + 7);
    const bool present = ((m >> slot) & 1ull) && !skipj;
    own[j] = present ? off0 + __popcll(m & ((1ull << slot) - 1ull)) : -1;
    outr[j] = (present && (ALL || !((xm >> slot) & 1ull))) ? own[j] : -1;
    // per face: the lane to take the value from (in-block), or the DOF to
    // load across the face (encoded as -2 - dof), or -1 (no neighbour)
#pragma unroll
    for (int f = 0; f < 2 * DIM; ++f) {
      int q[3] = {l[0], l[1], l[2]};
      q[f >> 1] += (f & 1) ? 1 : -1;
      const bool out = q[f >> 1] < 0 || q[f >> 1] >= G::BX;
      q[f >> 1] &= G::BX - 1;
      const int s2 = G::slot(q[0], q[1], q[2]);
      if (!out) {
        nsrc[j][f] = s2;
      } else {
        const unsigned long long fmk = lane_u64(lm, 8 * j + f + 1);
        const int fof = lane_i32(loff, 8 * j + f + 1);
        nsrc[j][f] = ((fmk >> s2) & 1ull) ? -2 - (fof + __popcll(fmk & ((1ull << s2) - 1ull)))
                                          : -1;
      }
    }
  }
  double d0 = 0.0, d1 = 0.0;
  for (int r = 0; r < (DOT ? 1 : nrhs); ++r) {
    const TA* ar = a + r * ld;
    TA aown[KB];
    double uv[KB], yv[KB], across[KB][2 * DIM];
#pragma unroll
    for (int j = 0; j < KB; ++j) {
      aown[j] = own[j] >= 0 ? ar[own[j]] : TA(0);
      uv[j] = (!ALL && outr[j] >= 0) ? (double)u[r * ld + outr[j]] : 0.0;
      yv[j] = (DOT && outr[j] >= 0) ? (double)dy[outr[j]] : 0.0;
#pragma unroll
      for (int f = 0; f < 2 * DIM; ++f)
        across[j][f] = (outr[j] >= 0 && nsrc[j][f] <= -2) ? (double)ar[-2 - nsrc[j][f]] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < KB; ++j) {
      double sum = 0.0;
#pragma unroll
      for (int f = 0; f < 2 * DIM; ++f) {
        const int src = nsrc[j][f] >= 0 ? nsrc[j][f] : slot;
        const double inb = (double)lane_take<TA>(aown[j], src);
        sum += nsrc[j][f] >= 0 ? inb : across[j][f];
      }
      if (outr[j] < 0) continue;
      double o = ALL ? coj[j] * sum : lap_out(cdj[j], uv[j], coj[j], sum);
      if (gsum) o += gscale * gsum[r];
      const TV ov = (TV)o;
      v[r * ld + outr[j]] = ov;
      if (DOT) {
        d0 += yv[j] * (double)ov;
        d1 += (double)ov * (double)ov;
      }
    }
  }
  if constexpr (DOT) wave_dot2(d0, d1, dpart, dnp, blockIdx.x * 4);
}

// Persistent and pipelined form of k_lap_sh for one right-hand side: each
// XCD takes a contiguous range of blocks and its wavefronts take every W-th
// block of it.  While block j is finished (cross-lane exchange, sums,
// store), the metadata of block j + 2 and the data of block j + 1 are
// already requested, so a wavefront keeps a block's loads in flight at all
// times.  (A wave's vector memory requests complete in issue order: each
// block's metadata is requested before the previous block's data, so
// waiting for it never waits for that data.)
template <int DIM>
struct LapIdx {
  int own, outr;    // DOF of the lane's slot (-1 absent); output DOF (-1 none)
  int xdof[DIM];    // per axis: DOF of the neighbour across the block face the
                    // lane lies on (-1 none, or the lane is on no face of it)
  int inst;         // instance of the block (composites), else 0
};
template <class TA, int DIM>
struct LapData {
  TA aown;
  double uv, yv;
  double across[DIM];
};

template <class TU, class TA, class TV, int DIM, bool ALL, bool DOT = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) void k_lap_pp(
    BlockView B, const TU* __restrict__ u, const TA* __restrict__ a, TV* __restrict__ v,
    double cd, double co, const double* __restrict__ gsum, double gscale,
    const double* __restrict__ coef, const int* __restrict__ skip,
    const TV* __restrict__ dy = nullptr, double* __restrict__ dpart = nullptr, int dnp = 0) {
  using G = Geo<DIM>;
  const int slot = threadIdx.x & 63;
  const int x = blockIdx.x & 7, W = (gridDim.x >> 3) * 4;
  const int wk = (blockIdx.x >> 3) * 4 + (threadIdx.x >> 6);
  const int q8 = B.nb >> 3, r8 = B.nb & 7;
  const int lo = x * q8 + (x < r8 ? x : r8), hi = lo + q8 + (x < r8 ? 1 : 0);
  const int l[3] = {G::lx(slot), G::ly(slot), G::lz(slot)};
  constexpr int step[3] = {1, G::BX, G::BX * G::BX};
  auto meta = [&](int blk, unsigned long long& lm, int& loff, int& lpad) {
    lm = 0ull;
    loff = lpad = 0;
    if (blk < hi && slot < 8) {
      const QMeta q = B.face[(int64_t)blk * 8 + slot];
      lm = q.mask;
      loff = q.off;
      lpad = q.pad;
    }
  };
  auto index = [&](unsigned long long lm, int loff, int lpad, LapIdx<DIM>& ix) {
    ix.inst = 0;
    bool skipj = false;
    if (coef) {
      const int inst = lane_i32(lpad, 7);
      ix.inst = inst > 0 ? inst : 0;
      skipj = skip && skip[ix.inst];
    }
    const unsigned long long m = lane_u64(lm, 0);
    const int off0 = lane_i32(loff, 0);
    const unsigned long long xm = lane_u64(lm, 7);
    const bool present = ((m >> slot) & 1ull) && !skipj;
    ix.own = present ? off0 + __popcll(m & ((1ull << slot) - 1ull)) : -1;
    ix.outr = (present && (ALL || !((xm >> slot) & 1ull))) ? ix.own : -1;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      // the lane lies on at most one face per axis: low (f = 2d) or high
      const bool low = l[d] == 0, high = l[d] == G::BX - 1;
      int q[3] = {l[0], l[1], l[2]};
      q[d] = low ? G::BX - 1 : 0;
      const int s2 = G::slot(q[0], q[1], q[2]);
      // readlane takes a wave-uniform lane: read both faces, select per lane
      const unsigned long long fm_lo = lane_u64(lm, 2 * d + 1), fm_hi = lane_u64(lm, 2 * d + 2);
      const int fo_lo = lane_i32(loff, 2 * d + 1), fo_hi = lane_i32(loff, 2 * d + 2);
      const unsigned long long fmk = low ? fm_lo : fm_hi;
      const int fof = low ? fo_lo : fo_hi;
      ix.xdof[d] = ((low || high) && ((fmk >> s2) & 1ull))
                       ? fof + __popcll(fmk & ((1ull << s2) - 1ull)) : -1;
    }
  };
  auto load = [&](const LapIdx<DIM>& ix, LapData<TA, DIM>& dt) {
    dt.aown = ix.own >= 0 ? a[ix.own] : TA(0);
    dt.uv = (!ALL && ix.outr >= 0) ? (double)u[ix.outr] : 0.0;
    dt.yv = (DOT && ix.outr >= 0) ? (double)dy[ix.outr] : 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d)
      dt.across[d] = (ix.outr >= 0 && ix.xdof[d] >= 0) ? (double)a[ix.xdof[d]] : 0.0;
  };
  double d0 = 0.0, d1 = 0.0;
  auto finish = [&](const LapIdx<DIM>& ix, const LapData<TA, DIM>& dt) {
    double sum = 0.0;
#pragma unroll
    for (int f = 0; f < 2 * DIM; ++f) {
      const int d = f >> 1;
      const bool out = (f & 1) ? l[d] == G::BX - 1 : l[d] == 0;
      const int src = out ? slot : slot + ((f & 1) ? step[d] : -step[d]);
      const double inb = (double)lane_take<TA>(dt.aown, src);
      sum += out ? dt.across[d] : inb;
    }
    if (ix.outr < 0) return;
    const double cdi = coef ? coef[2 * ix.inst] : cd;
    const double coi = coef ? coef[2 * ix.inst + 1] : co;
    double o = ALL ? coi * sum : lap_out(cdi, dt.uv, coi, sum);
    if (gsum) o += gscale * gsum[0];
    const TV ov = (TV)o;
    v[ix.outr] = ov;
    if (DOT) {
      d0 += dt.yv * (double)ov;
      d1 += (double)ov * (double)ov;
    }
  };
  int blk = lo + wk;
  if (blk < hi) {
    unsigned long long lm, lmn;
    int loff, lpad, loffn, lpadn;
    LapIdx<DIM> ic, in;
    LapData<TA, DIM> dc, dn;
    meta(blk, lm, loff, lpad);
    index(lm, loff, lpad, ic);
    meta(blk + W, lmn, loffn, lpadn);
    load(ic, dc);
    while (true) {
      const int nb = blk + W;
      const bool more = nb < hi;
      if (more) {
        index(lmn, loffn, lpadn, in);
        meta(nb + W, lmn, loffn, lpadn);
        load(in, dn);
      }
      finish(ic, dc);
      if (!more) break;
      ic = in;
      dc = dn;
      blk = nb;
    }
  }
  if constexpr (DOT) wave_dot2(d0, d1, dpart, dnp, blockIdx.x * 4);
}

// The Laplacian pass with its index arithmetic moved off the vector unit.
// Profiles of the pass forms above show them bound by vector-instruction
// issue, not by memory: about 250 vector instructions per block, almost all
// of them integer work on 64-bit masks (broadcasts of the metadata, prefix
// popcounts, bit tests).  Here a wavefront still handles one block, lane =
// slot, but
//   * the block's metadata (its own and its face neighbours' masks and first
//     DOFs, the explicit-row mask) is read with scalar loads: every mask is
//     wave-uniform and stays in scalar registers;
//   * lane sets (present slots, output rows, the lanes on a face whose
//     neighbour across it is present) are built with scalar mask arithmetic
//     and applied as execution masks (inverse ballot);
//   * a DOF is first DOF + the count of mask bits below the lane (two
//     masked-bit-count instructions), for the neighbour across a face on the
//     mask shifted by the face's slot offset;
//   * in-block neighbours' values come from other lanes: data-parallel
//     primitive moves inside 16-lane rows (x, and y in 3-D), lane permutes
//     across rows (z in 3-D, y in 2-D).
// The arithmetic and its order are those of k_lap_sh, so the outputs agree
// bit for bit.
template <class T>
__device__ __forceinline__ T lane_perm(T v, int addr) {
  if constexpr (sizeof(T) == 8) {
    const long long b = __double_as_longlong((double)v);
    const int lo = __builtin_amdgcn_ds_bpermute(addr, (int)(unsigned)(b & 0xffffffffll));
    const int hi = __builtin_amdgcn_ds_bpermute(addr, (int)(b >> 32));
    return (T)__longlong_as_double(((long long)hi << 32) | (unsigned)lo);
  } else {
    return __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int((float)v)));
  }
}
// value of lane (lane - k) (SHR) or (lane + k) (SHL) within a 16-lane row;
// lanes whose source lies outside their row get an unspecified value
template <class T, int CTRL>
__device__ __forceinline__ T lane_dpp(T v) {
  if constexpr (sizeof(T) == 8) {
    const long long b = __double_as_longlong((double)v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)(b & 0xffffffffll), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xf, 0xf, false);
    return (T)__longlong_as_double(((long long)hi << 32) | (unsigned)lo);
  } else {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int((float)v), CTRL, 0xf, 0xf, false));
  }
}
template <int K> constexpr int dpp_shr() { return 0x110 + K; }   // from lane - K
template <int K> constexpr int dpp_shl() { return 0x100 + K; }   // from lane + K


// lanes on the low and high face of the block along each axis (slots with
// local coordinate 0, or BX - 1, along it), evaluated at compile time
template <int DIM>
struct FaceLanes {
  unsigned long long lo[3], hi[3];
};
template <int DIM>
constexpr FaceLanes<DIM> face_lanes() {
  FaceLanes<DIM> f{{0ull, 0ull, 0ull}, {0ull, 0ull, 0ull}};
  constexpr int BX = DIM == 3 ? 4 : 8;
  for (int d = 0; d < DIM; ++d)
    for (int s = 0; s < 64; ++s) {
      const int l = DIM == 3 ? (d == 0 ? s & 3 : d == 1 ? (s >> 2) & 3 : s >> 4)
                             : (d == 0 ? s & 7 : s >> 3);
      if (l == 0) f.lo[d] |= 1ull << s;
      if (l == BX - 1) f.hi[d] |= 1ull << s;
    }
  return f;
}

constexpr int kLapWBlocksPerWave = 2;

template <class TU, class TA, class TV, int DIM, bool ALL, bool DOT = false>
__global__ __launch_bounds__(256) void k_lap_w(
    const QMeta* __restrict__ face, int nb, const TU* __restrict__ u, const TA* __restrict__ a,
    TV* __restrict__ v, int64_t ld, int nrhs, double cd, double co,
    const double* __restrict__ gsum, double gscale, int xcd, const double* __restrict__ coef,
    const int* __restrict__ skip, const TV* __restrict__ dy = nullptr,
    double* __restrict__ dpart = nullptr, int dnp = 0) {
  using G = Geo<DIM>;
  constexpr int BX = G::BX, KB = kLapWBlocksPerWave;
  constexpr int step[3] = {1, BX, BX * BX};
  constexpr FaceLanes<DIM> FL = face_lanes<DIM>();
  const int wg = xcd ? xcd_remap(blockIdx.x, gridDim.x) : blockIdx.x;
  const int blk0 = (wg * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6)) * KB;
  const int lane = threadIdx.x & 63;
  if (!DOT && blk0 >= nb) return;
  // per block j of the wave: coefficients, lane sets, DOFs (all but the DOFs
  // wave-uniform)
  double cdi[KB], coi[KB];
  unsigned long long present[KB], outm[KB], xload[KB][DIM];
  int own[KB], xdof[KB][DIM];
#pragma unroll
  for (int j = 0; j < KB; ++j) {
    const int blk = blk0 + j;
    cdi[j] = cd;
    coi[j] = co;
    present[j] = outm[j] = 0ull;
    own[j] = 0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      xload[j][d] = 0ull;
      xdof[j][d] = 0;
    }
    if (blk >= nb) continue;
    const QMeta* fb = face + (int64_t)blk * 8;
    const unsigned long long m = fb[0].mask;
    bool skipped = false;
    if (coef) {
      const int inst = fb[7].pad > 0 ? fb[7].pad : 0;
      cdi[j] = coef[2 * inst];
      coi[j] = coef[2 * inst + 1];
      skipped = skip && skip[inst];
    }
    present[j] = skipped ? 0ull : m;
    outm[j] = ALL ? present[j] : (present[j] & ~fb[7].mask);
    own[j] = lane_count_below(m, fb[0].off);
    // per axis: the DOF of the neighbour across the face the lane lies on,
    // and the lanes that load it (on that face, neighbour present, output row)
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const int K = (BX - 1) * step[d];
      const unsigned long long mlo = fb[2 * d + 1].mask, mhi = fb[2 * d + 2].mask;
      // low face: neighbour slot lane + K; high face: lane - K
      const unsigned long long slo = mlo >> K, shi = mhi << K;
      const int blo = fb[2 * d + 1].off + __popcll(mlo & ((1ull << K) - 1ull));
      const int dlo = lane_count_below(slo, blo), dhi = lane_count_below(shi, fb[2 * d + 2].off);
      xdof[j][d] = lane_in(FL.lo[d]) ? dlo : dhi;
      xload[j][d] = ((FL.lo[d] & slo) | (FL.hi[d] & shi)) & outm[j];
    }
  }
  const int zl = ((lane + step[DIM - 1]) & 63) << 2, zh = ((lane - step[DIM - 1]) & 63) << 2;
  double d0[KB], d1[KB];
#pragma unroll
  for (int j = 0; j < KB; ++j) d0[j] = d1[j] = 0.0;
  for (int r = 0; r < (DOT ? 1 : nrhs); ++r) {
    const TA* ar = a + r * ld;
    // every load of the wave's blocks first, then the exchanges and sums
    TA aown[KB];
    double uv[KB], yv[KB], across[KB][DIM];
#pragma unroll
    for (int j = 0; j < KB; ++j) {
      aown[j] = TA(0);
      uv[j] = yv[j] = 0.0;
      if (lane_in(present[j])) aown[j] = ar[own[j]];
      if (lane_in(outm[j])) {
        if (!ALL) uv[j] = (double)u[r * ld + own[j]];
        if (DOT) yv[j] = (double)dy[own[j]];
      }
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        across[j][d] = 0.0;
        if (lane_in(xload[j][d])) across[j][d] = (double)ar[xdof[j][d]];
      }
    }
#pragma unroll
    for (int j = 0; j < KB; ++j) {
      // in-block neighbours: low (-) and high (+) along each axis
      double lo[DIM], hi[DIM];
      lo[0] = (double)lane_dpp<TA, dpp_shr<1>()>(aown[j]);
      hi[0] = (double)lane_dpp<TA, dpp_shl<1>()>(aown[j]);
      if constexpr (DIM == 3) {
        lo[1] = (double)lane_dpp<TA, dpp_shr<4>()>(aown[j]);
        hi[1] = (double)lane_dpp<TA, dpp_shl<4>()>(aown[j]);
      }
      lo[DIM - 1] = (double)lane_perm<TA>(aown[j], zh);
      hi[DIM - 1] = (double)lane_perm<TA>(aown[j], zl);
      double sum = 0.0;
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        sum += lane_in(FL.lo[d]) ? across[j][d] : lo[d];
        sum += lane_in(FL.hi[d]) ? across[j][d] : hi[d];
      }
      if (lane_in(outm[j])) {
        double o = ALL ? coi[j] * sum : lap_out(cdi[j], uv[j], coi[j], sum);
        if (gsum) o += gscale * gsum[r];
        const TV ov = (TV)o;
        v[r * ld + own[j]] = ov;
        if (DOT) {
          d0[j] += yv[j] * (double)ov;
          d1[j] += (double)ov * (double)ov;
        }
      }
    }
  }
  // one partial per block (partial k = block k; slots past the last block
  // get zeros), so that the partials of a batch instance are the contiguous
  // range of its blocks
  if constexpr (DOT) {
#pragma unroll
    for (int j = 0; j < KB; ++j) {
      const double s0 = wave_sum(d0[j], 64), s1 = wave_sum(d1[j], 64);
      if (lane == 0) {
        dpart[blk0 + j] = s0;
        dpart[dnp + blk0 + j] = s1;
      }
    }
  }
}

template <class TS, bool DOT = false>
__global__ void k_lap_rows(int nrows, int nf, const int* __restrict__ row_id,
                           const int* __restrict__ col, const TS* __restrict__ u,
                           const double* __restrict__ a, TS* __restrict__ v, int64_t ld, int nrhs,
                           double cd, double co, const double* __restrict__ gsum, double gscale,
                           const double* __restrict__ coef, const int* __restrict__ row_inst,
                           const int* __restrict__ skip, const TS* __restrict__ dy = nullptr,
                           double* __restrict__ dpart = nullptr, int dnp = 0, int doff = 0) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double d0 = 0.0, d1 = 0.0;
  if (i < nrows && !(coef && skip && skip[row_inst[i]])) {
    const int id = row_id[i];
    if (coef) {
      cd = coef[2 * row_inst[i]];
      co = coef[2 * row_inst[i] + 1];
    }
    for (int r = 0; r < nrhs; ++r) {
      double s = 0.0;
      for (int f = 0; f < nf; ++f) {
        const int c = col[i * nf + f];
        if (c >= 0) s += a[r * ld + c];
      }
      double out = lap_out(cd, (double)u[r * ld + id], co, s);
      if (gsum) out += gscale * gsum[r];
      const TS ov = (TS)out;
      v[r * ld + id] = ov;
      if (DOT && r == 0) {
        d0 = (double)dy[id] * (double)ov;
        d1 = (double)ov * (double)ov;
      }
    }
  }
  // one partial per row (rows past the last one give zeros): a batch
  // instance's partials are the contiguous range of its explicit rows
  if (DOT) {
    dpart[doff + i] = d0;
    dpart[dnp + doff + i] = d1;
  }
}

// ---------------------------------------------------------------- gauge
// gsum[r] = sum_{i < n_s} u[r][i] (deterministic two-stage sum)
template <class T>
__global__ __launch_bounds__(256) void k_sum_part(const T* __restrict__ u, int64_t n_s, int64_t ld,
                                                  double* part) {
  __shared__ double s[256];
  const int r = blockIdx.y;
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n_s; i += (int64_t)gridDim.x * 256)
    acc += (double)u[r * ld + i];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[r * gridDim.x + blockIdx.x] = s[0];
}

__global__ void k_sum_final(const double* part, int np, double* out) {
  __shared__ double s[256];
  const int r = blockIdx.x;
  double acc = 0.0;
  for (int i = threadIdx.x; i < np; i += 256) acc += part[r * np + i];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[r] = s[0];
}

// ---------------------------------------------------------------- transpose
// E^T c for the tile rows of one parity class, one wavefront per tile.  The
// wave takes its tile and row range from one entry of the class table, so the
// tile's metadata and first row data are requested together, one load after
// it.  Rows go in chunks of kTRows: each lane of a chunk puts the stencil
// base of one row into LDS with the row's 1-D weights (the forward gather's
// FP64 weights), c_i folded into the last factor; then the wave walks the
// chunk's rows with one lane per stencil member (4 rows at a time in 2-D,
// where a stencil has 16 members), adding w c_i into the tile's (2 BX)^d cube
// in LDS.  A 3-D member's weight is the product of three 1-D weights read
// from LDS, and each lane sums over runs of rows with the same stencil base;
// 2-D uses LDS atomic adds (rows past the last one carry zero weights).  The
// cube is accumulated in FP64 for both precisions.  It is then added into z
// with plain loads and stores: tiles of one parity class stage disjoint
// blocks and the classes run as successive launches, so no two waves of a
// launch touch the same entry of z.  Chunks of 32 rows keep the LDS of a wave
// at 7.9 KB (20 waves per CU) where whole 64-row passes took 11.1 KB (14).
constexpr int kTRows = 32;
constexpr int kTGroup = 4;
template <class TS, int DIM>
__global__ __launch_bounds__(64) void k_gather_T(BlockView B, TileView tv, const int4* __restrict__ tbl,
                                                 int N, const double* __restrict__ c,
                                                 double* __restrict__ z, int64_t ld, int r,
                                                 int xcd) {
  using G = Geo<DIM>;
  constexpr int E = Cube<DIM>::E, EP = E + 1, NQ = 1 << DIM;
  constexpr int CS = DIM == 3 ? E * E * EP : E * EP;
  constexpr int M = DIM == 3 ? 64 : 16;       // stencil members
  constexpr int RPI = 64 / M;                 // rows per wave instruction
  constexpr int NW = DIM == 3 ? 12 : 8;       // 1-D weights per row
  constexpr int RC = kTRows;
  constexpr int RG = kTGroup;                 // rows whose LDS reads go out together
  static_assert(RC % 16 == 0 && RC <= 64 && RC % RG == 0, "chunk rows: a multiple of 16 and RG");
  __shared__ double s_z[CS];
  // per-row 1-D weights, component major; rows padded to RC + 1 entries so
  // that the four values of one component a wave reads for a row lie in
  // distinct LDS banks
  __shared__ double s_w[NW][RC + 1];
  __shared__ int s_b[RC];                     // per-row cube offset of member 0
  const int4 te = tbl[xcd ? xcd_remap(blockIdx.x, gridDim.x) : blockIdx.x];
  const int t = te.x, beg = te.y, end = te.z;
  if (beg == end) return;
  const int lane = threadIdx.x;
  unsigned long long qm = 0ull;
  int qoff = 0;
  if (lane < NQ) {
    const QMeta q = tv.meta[(int64_t)t * 8 + lane];
    qm = q.mask;
    qoff = q.off;
  }
  // entry of z (or -1) of this lane's node in staged block q, and its cube cell
  const int cx0 = G::lx(lane), cy0 = G::ly(lane), cz0 = G::lz(lane);
  auto zidx = [&](int q) {
    const unsigned long long m = lane_u64(qm, q);
    const int off = lane_i32(qoff, q);
    return ((m >> lane) & 1ull) ? off + __popcll(m & ((1ull << lane) - 1ull)) : -1;
  };
  auto cell = [&](int q) {
    const int qx = q & 1, qy = (q >> 1) & 1, qz = DIM == 3 ? (q >> 2) : 0;
    const int cx = qx * G::BX + cx0, cy = qy * G::BX + cy0, cz = qz * G::BX + cz0;
    return DIM == 3 ? (cz * E + cy) * EP + cx : cy * EP + cx;
  };
  // the old entries of z under the staged blocks, requested now so that the
  // loads overlap the row work (no other wave of this launch touches them);
  // the cube starts at zero and is added to them at the end
  double old[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int zi = zidx(q);
    old[q] = zi >= 0 ? z[r * ld + zi] : 0.0;
  }
  for (int idx = lane; idx < CS; idx += 64) s_z[idx] = 0.0;
  // this lane's stencil member and row slot within an instruction
  const int mo = lane & (M - 1), sub = lane / M;
  const int ma = mo & 3, mb = (mo >> 2) & 3, mc = DIM == 3 ? (mo >> 4) : 0;
  const int moff = DIM == 3 ? (mc * E + mb) * EP + ma : mb * EP + ma;
  // Row data of a chunk (lane < RC: row p0 + lane): local base, fraction
  // and c.  The next chunk's is requested before the current chunk's rows
  // are walked, and the DOFs (which c is read through) one chunk further
  // ahead, so only the first chunk waits for its loads.
  int lbn[3] = {0, 0, 0}, pmn = 0;
  double ttn[3] = {0.0, 0.0, 0.0}, cn = 0.0;
  if (lane < RC && beg + lane < end) {
    row_stencil<TS, DIM>(tv, beg + lane, lbn, ttn);
    cn = c[r * ld + tv.perm[beg + lane]];
  }
  if (lane < RC && beg + RC + lane < end) pmn = tv.perm[beg + RC + lane];
  for (int p0 = beg; p0 < end; p0 += RC) {
    const int nrow = min(RC, end - p0);
    const int lb[3] = {lbn[0], lbn[1], lbn[2]};
    const double tt[3] = {ttn[0], ttn[1], ttn[2]}, ci = cn;
    const int p1 = p0 + RC;
    if (lane < RC && p1 + lane < end) {
      row_stencil<TS, DIM>(tv, p1 + lane, lbn, ttn);
      cn = c[r * ld + pmn];
    }
    if (lane < RC && p1 + RC + lane < end) pmn = tv.perm[p1 + RC + lane];
    double wx[4] = {0.0, 0.0, 0.0, 0.0}, wy[4] = {0.0, 0.0, 0.0, 0.0};
    double wz[4] = {0.0, 0.0, 0.0, 0.0};
    int bs = 0;
    if (lane < nrow) {
      lagrange_p<double>(tv.p, tt[0], wx);
      lagrange_p<double>(tv.p, tt[1], wy);
      if (DIM == 3) {
        lagrange_p<double>(tv.p, tt[2], wz);
#pragma unroll
        for (int k = 0; k < 4; ++k) wz[k] *= ci;
      } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) wy[k] *= ci;
      }
      bs = DIM == 3 ? (lb[2] * E + lb[1]) * EP + lb[0] : lb[1] * EP + lb[0];
    }
    if (lane < RC) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        s_w[k][lane] = wx[k];
        s_w[4 + k][lane] = wy[k];
        if constexpr (DIM == 3) s_w[8 + k][lane] = wz[k];
      }
      s_b[lane] = bs;
    }
    __syncthreads();
    if constexpr (DIM == 3) {
      // Rows are sorted by stencil base, and runs of rows share one: each
      // lane sums its member's contributions in a register while the base
      // stays the same and adds the sum into the cube when it changes.  A
      // row's 64 members are distinct cells, and a wave's LDS operations
      // complete in order, so these read-add-writes need no atomics.
      double acc = 0.0;
      int cur = __builtin_amdgcn_readfirstlane(s_b[0]);
      for (int j = 0; j < nrow; j += RG) {
        // RG rows' bases and weights read at once (indices stay below RC)
        int bq[RG];
        double wq[RG];
#pragma unroll
        for (int u = 0; u < RG; ++u) {
          bq[u] = __builtin_amdgcn_readfirstlane(s_b[j + u]);
          wq[u] = (s_w[ma][j + u] * s_w[4 + mb][j + u]) * s_w[8 + mc][j + u];
        }
#pragma unroll
        for (int u = 0; u < RG; ++u) {
          if (j + u >= nrow) break;
          if (bq[u] != cur) {
            s_z[cur + moff] += acc;
            acc = 0.0;
            cur = bq[u];
          }
          acc += wq[u];
        }
      }
      s_z[cur + moff] += acc;
    } else {
      constexpr int UR = 4;                   // rows per lane per step
      const int nr = (nrow + UR * RPI - 1) / (UR * RPI) * (UR * RPI);
      for (int j0 = 0; j0 < nr; j0 += UR * RPI) {
        double v[UR];
        int o[UR];
#pragma unroll
        for (int u = 0; u < UR; ++u) {
          const int j = j0 + u * RPI + sub;
          v[u] = s_w[ma][j] * s_w[4 + mb][j];
          o[u] = s_b[j] + moff;
        }
#pragma unroll
        for (int u = 0; u < UR; ++u) atomicAdd(&s_z[o[u]], v[u]);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int zi = zidx(q);
    if (zi >= 0) z[r * ld + zi] = old[q] + s_z[cell(q)];
  }
}

// E^T c over the explicit rows by pull lists: one wavefront per target DOF
// (four per workgroup).  The lanes take the target's contiguous segment of
// entries 64 at a time (entry e: weight w[e] of source row src[e], FP64 for
// both precisions), sum the products w c_src in their own order and the wave
// adds the tree sum of its lanes into z once: the same value on every run,
// with no atomics.
__global__ __launch_bounds__(256) void k_et_pull(int n_tgt, const int* __restrict__ tgt,
                                                 const int* __restrict__ start,
                                                 const int* __restrict__ src,
                                                 const double* __restrict__ w,
                                                 const double* __restrict__ c,
                                                 double* __restrict__ z) {
  const int k = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (k >= n_tgt) return;                     // whole waves leave together
  const int lane = threadIdx.x & 63;
  const int b0 = start[k], b1 = start[k + 1];
  double acc = 0.0;
  for (int e = b0 + lane; e < b1; e += 64) acc += w[e] * c[src[e]];
  acc = wave_sum(acc, 64);
  if (lane == 0) z[tgt[k]] += acc;
}

// The corrections of (L - diag L)^T w for explicit FD rows by pull lists:
// c[t] += co (sum of +w_i over rows adding to t, -w_i over swapped rows
// moving their entry away from t), in ascending source order.
template <class TS>
__global__ void k_lt_pull(int n_tgt, const int* __restrict__ tgt, const int* __restrict__ start,
                          const int* __restrict__ src, const int* __restrict__ row_id,
                          const TS* __restrict__ w, double* __restrict__ c, int64_t ld, int nrhs,
                          double co) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_tgt) return;
  const int t = tgt[k], b0 = start[k], b1 = start[k + 1];
  for (int r = 0; r < nrhs; ++r) {
    double acc = 0.0;
    for (int e = b0; e < b1; ++e) {
      const int v = src[e];
      const double wi = co * (double)w[r * ld + row_id[v >> 1]];
      acc += (v & 1) ? -wi : wi;
    }
    c[r * ld + t] += acc;
  }
}

template <class T>
__global__ void k_fill(T* __restrict__ p, int64_t n, T val) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = val;
}

// out = cd w + nn e (FP64 arithmetic, stored in the vector precision TS);
// with DOT also the partials of (dy, out) and (out, out)
template <class TS, bool DOT = false>
__global__ void k_combine(const TS* __restrict__ w, const double* __restrict__ z,
                          TS* __restrict__ out, double cd, double nn, int64_t total,
                          const TS* __restrict__ dy = nullptr, double* __restrict__ dpart = nullptr,
                          int dnp = 0) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double d0 = 0.0, d1 = 0.0;
  if (i < total) {
    const TS o = (TS)(cd * (double)w[i] + nn * z[i]);
    out[i] = o;
    if (DOT) {
      d0 = (double)dy[i] * (double)o;
      d1 = (double)o * (double)o;
    }
  }
  if (DOT) wave_dot2(d0, d1, dpart, dnp, blockIdx.x * 4);
}

// ---------------------------------------------------------------- rhs
__global__ void k_rhs_init(int64_t n_s, int64_t n_c, int nrhs, const double* __restrict__ f,
                           const int* __restrict__ bc_node, double* __restrict__ b) {
  const int64_t n = n_s + n_c;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * nrhs) return;
  const int64_t r = t / n, i = t % n;
  b[t] = i < n_s ? f[r * n_s + i] : f[r * n_s + bc_node[i - n_s]];
}

__global__ void k_rhs_rows(int nrows, int nf, int64_t n_s, int64_t n_c, int nrhs,
                           const int* __restrict__ row_id, const int* __restrict__ col,
                           const double* __restrict__ g, const double* __restrict__ ecoef,
                           double scale, double* __restrict__ b) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nrows) return;
  const int id = row_id[i];
  const int64_t n = n_s + n_c;
  for (int r = 0; r < nrhs; ++r) {
    double s = 0.0;
    for (int f = 0; f < nf; ++f) {
      const int c = col[i * nf + f];
      if (c >= n_s) s += ecoef[c - n_s] * g[r * n_c + (c - n_s)];
    }
    b[r * n + id] -= scale * s;
  }
}

__global__ void k_gradf(int64_t n_s, int64_t n_c, int nrhs, const double* __restrict__ lam,
                        double* __restrict__ gf) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_s * nrhs) return;
  const int64_t r = t / n_s, i = t % n_s;
  gf[t] = lam[r * (n_s + n_c) + i];
}

__global__ void k_gradf_bc(int64_t n_s, int64_t n_c, int nrhs, const int* __restrict__ bc_node,
                           const double* __restrict__ lam, double* __restrict__ gf) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_c * nrhs) return;
  const int64_t r = t / n_c, k = t % n_c;
  gf[r * n_s + bc_node[k]] += lam[r * (n_s + n_c) + n_s + k];
}

__global__ void k_gradg(int nrows, int nf, int64_t n_s, int64_t n_c, int nrhs,
                        const int* __restrict__ row_id, const int* __restrict__ col,
                        const double* __restrict__ lam, const double* __restrict__ ecoef,
                        double scale, double* __restrict__ gg) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nrows) return;
  const int id = row_id[i];
  const int64_t n = n_s + n_c;
  for (int r = 0; r < nrhs; ++r) {
    const double li = lam[r * n + id];
    for (int f = 0; f < nf; ++f) {
      const int c = col[i * nf + f];
      if (c >= n_s && ecoef[c - n_s] != 0.0)
        atomicAdd(&gg[r * n_c + (c - n_s)], scale * ecoef[c - n_s] * li);
    }
  }
}

// ================================================================ host
template <class T>
static const Tune& tune_of(const cpm_band* b) {
  return b->tune[sizeof(T) == 8 ? 0 : 1];
}

template <class T, int DIM, int PAD>
static void launch_gather_k(const cpm_band* b, int k, const T* ur, double* ar, int64_t ld,
                            int xcd, int ps, hipStream_t st, const int* skip) {
  const dim3 g(b->ntiles), t(64);
  TileView tvs = tview(b);
  tvs.skip = skip;
  if (ps == 2 && !b->tile_inst) {
    int64_t gp = ((int64_t)b->ntiles + 7) / 8 * 8;
    if (gp > 8 * (int64_t)kPersistWavesPerXcd) gp = 8 * (int64_t)kPersistWavesPerXcd;
    const dim3 gq((unsigned)gp);
    switch (k) {
      case 1: hipLaunchKernelGGL((k_gather_pp<T, DIM, 1, PAD>), gq, t, 0, st, bview(b), tview(b), b->N, ur, ar, ld, b->ntiles); break;
      case 2: hipLaunchKernelGGL((k_gather_pp<T, DIM, 2, PAD>), gq, t, 0, st, bview(b), tview(b), b->N, ur, ar, ld, b->ntiles); break;
      case 3: hipLaunchKernelGGL((k_gather_pp<T, DIM, 3, PAD>), gq, t, 0, st, bview(b), tview(b), b->N, ur, ar, ld, b->ntiles); break;
      default: hipLaunchKernelGGL((k_gather_pp<T, DIM, 4, PAD>), gq, t, 0, st, bview(b), tview(b), b->N, ur, ar, ld, b->ntiles); break;
    }
    CPM_LAUNCH_CHECK();
    return;
  }
  if (ps && !b->tile_inst) {
    // a multiple of 8 wavefronts: every XCD gets the same number
    int64_t gp = ((int64_t)b->ntiles + 7) / 8 * 8;
    if (gp > 8 * (int64_t)kPersistWavesPerXcd) gp = 8 * (int64_t)kPersistWavesPerXcd;
    const dim3 gq((unsigned)gp);
    switch (k) {
      case 1: hipLaunchKernelGGL((k_gather_ps<T, DIM, 1, PAD>), gq, t, 0, st, bview(b), tview(b), b->N, ur, ar, ld, b->ntiles); break;
      case 2: hipLaunchKernelGGL((k_gather_ps<T, DIM, 2, PAD>), gq, t, 0, st, bview(b), tview(b), b->N, ur, ar, ld, b->ntiles); break;
      case 3: hipLaunchKernelGGL((k_gather_ps<T, DIM, 3, PAD>), gq, t, 0, st, bview(b), tview(b), b->N, ur, ar, ld, b->ntiles); break;
      default: hipLaunchKernelGGL((k_gather_ps<T, DIM, 4, PAD>), gq, t, 0, st, bview(b), tview(b), b->N, ur, ar, ld, b->ntiles); break;
    }
    CPM_LAUNCH_CHECK();
    return;
  }
  if (b->p == 2) {
    switch (k) {
      case 1: hipLaunchKernelGGL((k_gather<T, DIM, 1, PAD, 3>), g, t, 0, st, bview(b), tvs, b->N, ur, ar, ld, xcd); break;
      case 2: hipLaunchKernelGGL((k_gather<T, DIM, 2, PAD, 3>), g, t, 0, st, bview(b), tvs, b->N, ur, ar, ld, xcd); break;
      case 3: hipLaunchKernelGGL((k_gather<T, DIM, 3, PAD, 3>), g, t, 0, st, bview(b), tvs, b->N, ur, ar, ld, xcd); break;
      default: hipLaunchKernelGGL((k_gather<T, DIM, 4, PAD, 3>), g, t, 0, st, bview(b), tvs, b->N, ur, ar, ld, xcd); break;
    }
    CPM_LAUNCH_CHECK();
    return;
  }
  switch (k) {
    case 1: hipLaunchKernelGGL((k_gather<T, DIM, 1, PAD>), g, t, 0, st, bview(b), tvs, b->N, ur, ar, ld, xcd); break;
    case 2: hipLaunchKernelGGL((k_gather<T, DIM, 2, PAD>), g, t, 0, st, bview(b), tvs, b->N, ur, ar, ld, xcd); break;
    case 3: hipLaunchKernelGGL((k_gather<T, DIM, 3, PAD>), g, t, 0, st, bview(b), tvs, b->N, ur, ar, ld, xcd); break;
    default: hipLaunchKernelGGL((k_gather<T, DIM, 4, PAD>), g, t, 0, st, bview(b), tvs, b->N, ur, ar, ld, xcd); break;
  }
  CPM_LAUNCH_CHECK();
}

template <class T, int DIM>
static void launch_gather(const cpm_band* b, int nrhs, const T* u, double* a, hipStream_t st,
                          hipEvent_t* ev, const int* skip) {
  const int64_t ld = b->n;
  int r = 0;
  while (r < nrhs) {
    const int k = nrhs - r >= 4 ? 4 : nrhs - r;
    const T* ur = u + r * ld;
    double* ar = a + r * ld;
    if (b->ntiles) {
      const Tune& tn = tune_of<T>(b);
      if (tn.pad) launch_gather_k<T, DIM, 4>(b, k, ur, ar, ld, tn.xcd, tn.ps, st, skip);
      else launch_gather_k<T, DIM, 1>(b, k, ur, ar, ld, tn.xcd, tn.ps, st, skip);
    }
    r += k;
  }
  if (ev) CPM_HIP(hipEventRecord(ev[1], st));
  if (b->n_erows) {
    const int nm = DIM == 3 ? 64 : 16;
    hipLaunchKernelGGL(k_gather_rows<T>, dim3(grid_for((int64_t)b->n_erows * nm, 256)), dim3(256),
                       0, st, b->n_erows, nm, b->erow_id, b->ecol, b->ew, u, a, ld, nrhs,
                       b->erow_inst, skip);
    CPM_LAUNCH_CHECK();
  }
  if (ev) CPM_HIP(hipEventRecord(ev[2], st));
}

// Workgroups (4 wavefronts each) of the Laplacian pass in the tuned form; the
// persistent form (lap 2) launches at most kLapPersistWGsPerXcd per XCD.
constexpr int kLapPersistWGsPerXcd = 384;
static int lap_groups(const cpm_band* b, const Tune& tn) {
  if (tn.lap == 2) {
    int g = (b->nb + 31) / 32 * 8;   // a multiple of 8: every XCD gets as many
    if (g > 8 * kLapPersistWGsPerXcd) g = 8 * kLapPersistWGsPerXcd;
    return g < 8 ? 8 : g;
  }
  const int kb = tn.lap == 3 ? kLapWBlocksPerWave : tn.lap ? kLapShBlocksPerWave : kLapBlocksPerWave;
  return (b->nb + 4 * kb - 1) / (4 * kb);
}
static int lap_row_groups(const cpm_band* b) {
  return b->n_lrows ? grid_for(b->n_lrows, 128) : 0;
}

// Partials of a fused dot product written by the Laplacian pass (per value):
// one per wavefront, or one per block slot for k_lap_w (lap 3).
static int lap_dot_parts(const cpm_band* b, const Tune& tn) {
  if (b->composite && tn.lap != 3) {   // composites take fused dots in lap 3 only
    Tune t3 = tn;
    t3.lap = 3;
    return lap_dot_parts(b, t3);
  }
  return 4 * lap_groups(b, tn) * (tn.lap == 3 ? kLapWBlocksPerWave : 1);
}

// Number of partials a fused dot product of an apply writes (per value): those
// of the Laplacian pass, for the launch variant the band is tuned to in that
// precision, then one per thread of the explicit FD rows' kernel.
int apply_dot_parts(const cpm_band* b, bool transpose, bool f32) {
  if (transpose) return 4 * grid_for(b->n, 256);
  return lap_dot_parts(b, b->tune[f32 ? 1 : 0]) + 128 * lap_row_groups(b);
}

// The Laplacian pass in the band's tuned form (k_lap or k_lap_sh).
template <class TU, class TA, class TV, int DIM, bool ALL, bool DOT>
static void launch_lap(const cpm_band* b, const Tune& tn, hipStream_t st, const TU* u,
                       const TA* a, TV* v, int64_t ld, int nrhs, double cd, double co,
                       const double* gsum, double gscale, const double* coef, const int* skip,
                       const TV* dy, double* dpart, int dnp) {
  if (DOT && b->composite && tn.lap != 3) {
    // a batch finishes each system's dot products over its own blocks'
    // partials, which only k_lap_w writes per block
    Tune t3 = tn;
    t3.lap = 3;
    launch_lap<TU, TA, TV, DIM, ALL, DOT>(b, t3, st, u, a, v, ld, nrhs, cd, co, gsum, gscale,
                                          coef, skip, dy, dpart, dnp);
    return;
  }
  if (tn.lap == 2 && nrhs > 1) {   // the persistent form takes one right-hand side
    Tune t1 = tn;
    t1.lap = 1;
    launch_lap<TU, TA, TV, DIM, ALL, DOT>(b, t1, st, u, a, v, ld, nrhs, cd, co, gsum, gscale,
                                          coef, skip, dy, dpart, dnp);
    return;
  }
  const dim3 g(lap_groups(b, tn)), t(256);
  if (tn.lap == 3)
    hipLaunchKernelGGL((k_lap_w<TU, TA, TV, DIM, ALL, DOT>), g, t, 0, st, b->blk_face, b->nb, u,
                       a, v, ld, nrhs, cd, co, gsum, gscale, tn.xcd, coef, skip, dy, dpart, dnp);
  else if (tn.lap == 2)
    hipLaunchKernelGGL((k_lap_pp<TU, TA, TV, DIM, ALL, DOT>), g, t, 0, st, bview(b), u, a, v, cd,
                       co, gsum, gscale, coef, skip, dy, dpart, dnp);
  else if (tn.lap)
    hipLaunchKernelGGL((k_lap_sh<TU, TA, TV, DIM, ALL, DOT>), g, t, 0, st, bview(b), u, a, v, ld,
                       nrhs, cd, co, gsum, gscale, tn.xcd, coef, skip, dy, dpart, dnp);
  else
    hipLaunchKernelGGL((k_lap<TU, TA, TV, DIM, ALL, DOT>), g, t, 0, st, bview(b), u, a, v, ld,
                       nrhs, cd, co, gsum, gscale, tn.xcd, coef, skip, dy, dpart, dnp);
  CPM_LAUNCH_CHECK();
}

// Bytes of scratch one forward apply of nrhs right-hand sides needs: the
// intermediate a = E u, FP64 for both vector precisions.
size_t apply_scratch_bytes(const cpm_band* b, int nrhs) {
  return sizeof(double) * (size_t)b->n * (size_t)nrhs;
}

// The two passes of the forward apply with a given scratch vector a (at
// least apply_scratch_bytes).  ev (optional): five events recorded between
// the four phases.
template <class T, int DIM>
static void apply_dim_one(const cpm_band* b, double m, double n, const T* u, T* v, hipStream_t st,
                          double* a, const int* skip, int nrhs = 1, const double* gsum = nullptr,
                          double gamma = 0.0, hipEvent_t* ev = nullptr, const T* dy = nullptr,
                          double* dpart = nullptr);

template <class T, int DIM>
static void apply_dim(const cpm_band* b, double m, double n, int nrhs, const T* u, T* v,
                      hipStream_t st, const double* gsum, double gamma, double* a,
                      hipEvent_t* ev = nullptr, const T* dy = nullptr, double* dpart = nullptr) {
  const int64_t ld = b->n;
  // A batch composite applies each right-hand side in launches of its own,
  // so that the kernels skip every converged system, not only instances
  // whose systems have all converged (skip flags [nrhs][instances]).
  // With fused dot products, right-hand side r writes its partials to
  // dpart + 2 r apply_dot_parts.
  if (b->composite && nrhs > 1 && !ev && !gsum) {
    const int np = apply_dot_parts(b, false, sizeof(T) == 4);
    for (int r = 0; r < nrhs; ++r)
      apply_dim_one<T, DIM>(b, m, n, u + r * ld, v + r * ld, st, a + r * ld,
                            b->inst_skip ? b->inst_skip + (size_t)r * b->skip_stride : nullptr,
                            1, nullptr, 0.0, nullptr, dy ? dy + r * ld : nullptr,
                            dy ? dpart + (size_t)2 * r * np : nullptr);
    return;
  }
  apply_dim_one<T, DIM>(b, m, n, u, v, st, a, b->inst_skip, nrhs, gsum, gamma, ev, dy, dpart);
}

template <class T, int DIM>
static void apply_dim_one(const cpm_band* b, double m, double n, const T* u, T* v, hipStream_t st,
                          double* a, const int* skip, int nrhs, const double* gsum, double gamma,
                          hipEvent_t* ev, const T* dy, double* dpart) {
  const int64_t ld = b->n;
  if (ev) CPM_HIP(hipEventRecord(ev[0], st));
  launch_gather<T, DIM>(b, nrhs, u, a, st, ev, skip);
  const double N2 = (double)b->N * (double)b->N;
  const double cd = m + n * (-2.0 * DIM * N2);
  const double co = n * N2;
  const double gscale = gsum ? gamma / (double)b->n_s : 0.0;
  const int g1 = lap_dot_parts(b, tune_of<T>(b)), g2 = lap_row_groups(b), np = g1 + 128 * g2;
  if (dy)
    launch_lap<T, double, T, DIM, false, true>(b, tune_of<T>(b), st, u, a, v, ld, nrhs, cd, co,
                                               gsum, gscale, b->inst_coef, skip, dy,
                                               dpart, np);
  else
    launch_lap<T, double, T, DIM, false, false>(b, tune_of<T>(b), st, u, a, v, ld, nrhs, cd, co,
                                                gsum, gscale, b->inst_coef, skip,
                                                nullptr, nullptr, 0);
  if (ev) CPM_HIP(hipEventRecord(ev[3], st));
  if (b->n_lrows) {
    if (dy)
      hipLaunchKernelGGL((k_lap_rows<T, true>), dim3(g2), dim3(128), 0, st, b->n_lrows, 2 * DIM,
                         b->lrow_id, b->lcol, u, a, v, ld, nrhs, cd, co, gsum, gscale,
                         b->inst_coef, b->lrow_inst, skip, dy, dpart, np, g1);
    else
      hipLaunchKernelGGL((k_lap_rows<T>), dim3(g2), dim3(128), 0, st, b->n_lrows, 2 * DIM,
                         b->lrow_id, b->lcol, u, a, v, ld, nrhs, cd, co, gsum, gscale,
                         b->inst_coef, b->lrow_inst, skip, nullptr, nullptr, 0, 0);
    CPM_LAUNCH_CHECK();
  }
  if (ev) CPM_HIP(hipEventRecord(ev[4], st));
}

template <class T>
void apply_with_scratch(const cpm_band* b, double m, double n, int nrhs, const T* u, T* v,
                        hipStream_t st, double* a, hipEvent_t* ev) {
  if (b->dim == 3) apply_dim<T, 3>(b, m, n, nrhs, u, v, st, nullptr, 0.0, a, ev);
  else apply_dim<T, 2>(b, m, n, nrhs, u, v, st, nullptr, 0.0, a, ev);
}

template <class T>
void apply_impl(const cpm_band* b, double m, double n, int nrhs, const T* u, T* v, hipStream_t st,
                const double* gauge_sum, double gamma, const T* dy, double* dpart) {
  double* gs = nullptr;
  if (gamma != 0.0) {
    // gauge: gamma * (sum of the PDE entries of u) / n_s on every row
    const int np = 256;
    double* part = static_cast<double*>(band_scratch(b, 3, sizeof(double) * np * nrhs + 64));
    gs = gauge_sum ? const_cast<double*>(gauge_sum)
                   : static_cast<double*>(band_scratch(b, 4, sizeof(double) * nrhs + 64));
    hipLaunchKernelGGL(k_sum_part<T>, dim3(np, nrhs), dim3(256), 0, st, u, b->n_s, b->n, part);
    CPM_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_sum_final, dim3(nrhs), dim3(256), 0, st, part, np, gs);
    CPM_LAUNCH_CHECK();
  }
  double* a = static_cast<double*>(band_scratch(b, 0, apply_scratch_bytes(b, nrhs)));
  if (b->dim == 3) apply_dim<T, 3>(b, m, n, nrhs, u, v, st, gs, gamma, a, nullptr, dy, dpart);
  else apply_dim<T, 2>(b, m, n, nrhs, u, v, st, gs, gamma, a, nullptr, dy, dpart);
}

// The transposed apply.  c = (L - diag L)^T w and e = E^T c are FP64 scratch
// vectors for both storage precisions (the combine step cancels the two
// terms of size N^2, as the forward Laplacian pass does).
template <class T, int DIM>
static void apply_T_dim(const cpm_band* b, double m, double n, int nrhs, const T* w, T* z,
                        hipStream_t st, const T* dy = nullptr, double* dpart = nullptr) {
  const int64_t ld = b->n;
  double* c = static_cast<double*>(band_scratch(b, 1, sizeof(double) * (size_t)ld * nrhs));
  double* e = static_cast<double*>(band_scratch(b, 2, sizeof(double) * (size_t)ld * nrhs));
  const double N2 = (double)b->N * (double)b->N;
  const double co = N2;
  // c = (L - diag L)^T w: symmetric bulk over every PDE row, then corrections
  // (fill kernels, not memsets: this sequence may be captured into a graph);
  // k_lap<ALL> writes every PDE entry, so only the BC entries need clearing
  if (b->n_c)
    for (int r = 0; r < nrhs; ++r)
      hipLaunchKernelGGL(k_fill<double>, dim3(grid_for(b->n_c, 256, 4096)), dim3(256), 0, st,
                         c + r * ld + b->n_s, (int64_t)b->n_c, 0.0);
  launch_lap<T, T, double, DIM, true, false>(b, tune_of<T>(b), st, w, w, c, ld, nrhs, 0.0, co,
                                             nullptr, 0.0, nullptr, nullptr, nullptr, nullptr, 0);
  if (b->lt_tgt) {
    if (b->n_lt) {
      hipLaunchKernelGGL(k_lt_pull<T>, dim3(grid_for(b->n_lt, 256)), dim3(256), 0, st, b->n_lt,
                         b->lt_tgt, b->lt_start, b->lt_src, b->lrow_id, w, c, ld, nrhs, co);
      CPM_LAUNCH_CHECK();
    }
  } else if (b->n_lrows) {
    CPM_FAIL(CPM_E_INVALID, "this band has no transposed FD pull lists");
  }
  // e = E^T c
  hipLaunchKernelGGL(k_fill<double>, dim3(grid_for(ld * nrhs, 256, 4096)), dim3(256), 0, st, e,
                     ld * nrhs, 0.0);
  if (b->ntiles) {
    if (!b->tile_col) CPM_FAIL(CPM_E_INVALID, "this band has no transpose schedule");
    for (int r = 0; r < nrhs; ++r)
      for (int k = 0; k < 8; ++k) {
        const int cnt = b->col_start[k + 1] - b->col_start[k];
        if (!cnt) continue;
        hipLaunchKernelGGL((k_gather_T<T, DIM>), dim3(cnt), dim3(64), 0, st, bview(b), tview(b),
                           b->tile_col + b->col_start[k], b->N, c, e, ld, r, tune_of<T>(b).xcd);
        CPM_LAUNCH_CHECK();
      }
  }
  if (b->et_tgt) {
    if (b->n_et) {
      for (int r = 0; r < nrhs; ++r)
        hipLaunchKernelGGL(k_et_pull, dim3((b->n_et + 3) / 4), dim3(256), 0, st, b->n_et,
                           b->et_tgt, b->et_start, b->et_src, b->et_w, c + r * ld, e + r * ld);
      CPM_LAUNCH_CHECK();
    }
  } else if (b->n_erows) {
    CPM_FAIL(CPM_E_INVALID, "this band has no transposed interpolation pull lists");
  }
  const double cd = m + n * (-2.0 * DIM * N2);
  const int64_t total = ld * nrhs;
  const int gc = grid_for(total, 256);
  if (dy) {
    if ((int64_t)gc * 256 < total) CPM_FAIL(CPM_E_INVALID, "internal: fused dot grid too small");
    hipLaunchKernelGGL((k_combine<T, true>), dim3(gc), dim3(256), 0, st, w, e, z, cd, n, total,
                       dy, dpart, 4 * gc);
  } else {
    hipLaunchKernelGGL((k_combine<T>), dim3(gc), dim3(256), 0, st, w, e, z, cd, n, total,
                       nullptr, nullptr, 0);
  }
  CPM_LAUNCH_CHECK();
}

template <class T>
void apply_transpose_impl(const cpm_band* b, double m, double n, int nrhs, const T* w, T* z,
                          hipStream_t st, const double*, double gamma, const T* dy,
                          double* dpart) {
  if (gamma != 0.0) CPM_FAIL(CPM_E_INVALID, "the gauge is not supported for the transpose");
  if (b->dim == 3) apply_T_dim<T, 3>(b, m, n, nrhs, w, z, st, dy, dpart);
  else apply_T_dim<T, 2>(b, m, n, nrhs, w, z, st, dy, dpart);
}

template void apply_impl<double>(const cpm_band*, double, double, int, const double*, double*,
                                 hipStream_t, const double*, double, const double*, double*);
template void apply_impl<float>(const cpm_band*, double, double, int, const float*, float*,
                                hipStream_t, const double*, double, const float*, double*);
template void apply_transpose_impl<double>(const cpm_band*, double, double, int, const double*,
                                           double*, hipStream_t, const double*, double,
                                           const double*, double*);
template void apply_transpose_impl<float>(const cpm_band*, double, double, int, const float*,
                                          float*, hipStream_t, const double*, double,
                                          const float*, double*);

}  // namespace cpm

using namespace cpm;

static void check_vec_args(const cpm_band* b, int dtype, int nrhs, const void* x, const void* y) {
  if (!b) CPM_FAIL(CPM_E_INVALID, "null band");
  if (dtype != CPM_F64 && dtype != CPM_F32) CPM_FAIL(CPM_E_INVALID, "unknown dtype %d", dtype);
  if (nrhs < 1) CPM_FAIL(CPM_E_INVALID, "nrhs must be >= 1 (got %d)", nrhs);
  if ((int64_t)nrhs * b->n >= (1ll << 31))
    CPM_FAIL(CPM_E_INVALID, "nrhs * n exceeds the 32-bit index range");
  if (!x || !y) CPM_FAIL(CPM_E_INVALID, "null vector");
  if (x == y) CPM_FAIL(CPM_E_INVALID, "input and output must not alias");
}

extern "C" cpm_status cpm_apply(const cpm_band* b, double m, double n, int dtype, int nrhs,
                                const void* u, void* v, void* hip_stream) {
  return guard([&] {
    check_vec_args(b, dtype, nrhs, u, v);
    hipStream_t st = (hipStream_t)hip_stream;
    if (dtype == CPM_F64)
      apply_impl<double>(b, m, n, nrhs, (const double*)u, (double*)v, st);
    else
      apply_impl<float>(b, m, n, nrhs, (const float*)u, (float*)v, st);
  });
}

// ---------------------------------------------------------------- no-alloc
// cpm_apply for callers that cannot allocate device memory.  The scratch the
// apply needs (the FP64 intermediate a = E u) lives in a file-scope device
// array of kNoAllocScratchBytes, one copy per GPU the library runs on, held
// until the process ends.  Host code never passes the array's name to a
// kernel (on the host it only stands in for the symbol): its device address
// is looked up once per device with hipGetSymbolAddress and kept in
// g_noalloc_ptr.  Calls on one GPU share the array, so calls that overlap on
// one GPU (different streams, or threads) race on it.  Every entry of a the
// apply reads is written by the same apply first, so nothing needs clearing.
constexpr size_t kNoAllocScratchBytes = size_t(32) << 20;   // 32 MiB
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[kMaxDevices] = {};

void* noalloc_scratch() {
  int dev = 0;
  CPM_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) CPM_FAIL(CPM_E_INVALID, "device ordinal %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* ptr = nullptr;
    CPM_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) CPM_FAIL(CPM_E_HIP, "hipGetSymbolAddress returned a null scratch address");
    g_noalloc_ptr[dev] = ptr;
  }
  return g_noalloc_ptr[dev];
}
}  // namespace

extern "C" cpm_status cpm_apply_noalloc(const cpm_band* b, double m, double n, int dtype,
                                        int nrhs, const void* u, void* v, void* hip_stream) {
  return guard([&] {
    check_vec_args(b, dtype, nrhs, u, v);
    const size_t need = apply_scratch_bytes(b, nrhs);
    if (need > kNoAllocScratchBytes)
      CPM_FAIL(CPM_E_INVALID,
               "cpm_apply_noalloc: n * nrhs = %lld needs %zu bytes of scratch, above the "
               "%zu-byte static limit (n * nrhs <= %zu); use cpm_apply",
               (long long)(b->n * nrhs), need, kNoAllocScratchBytes,
               kNoAllocScratchBytes / sizeof(double));
    double* a = static_cast<double*>(noalloc_scratch());
    hipStream_t st = (hipStream_t)hip_stream;
    if (dtype == CPM_F64)
      apply_with_scratch<double>(b, m, n, nrhs, (const double*)u, (double*)v, st, a, nullptr);
    else
      apply_with_scratch<float>(b, m, n, nrhs, (const float*)u, (float*)v, st, a, nullptr);
  });
}

extern "C" cpm_status cpm_apply_profile(const cpm_band* b, double m, double n, int dtype,
                                        int nrhs, const void* u, void* v, int reps,
                                        void* hip_stream, double* ms) {
  return guard([&] {
    check_vec_args(b, dtype, nrhs, u, v);
    if (reps < 1 || !ms) CPM_FAIL(CPM_E_INVALID, "reps must be >= 1 and ms non-null");
    hipStream_t st = (hipStream_t)hip_stream;
    hipEvent_t ev[5];
    for (auto& e : ev) CPM_HIP(hipEventCreate(&e));
    double acc[4] = {0, 0, 0, 0};
    try {
      for (int k = 0; k < reps; ++k) {
        double* a = static_cast<double*>(band_scratch(b, 0, apply_scratch_bytes(b, nrhs)));
        if (dtype == CPM_F64)
          apply_with_scratch<double>(b, m, n, nrhs, (const double*)u, (double*)v, st, a, ev);
        else
          apply_with_scratch<float>(b, m, n, nrhs, (const float*)u, (float*)v, st, a, ev);
        CPM_HIP(hipEventSynchronize(ev[4]));
        for (int p = 0; p < 4; ++p) {
          float t = 0.f;
          CPM_HIP(hipEventElapsedTime(&t, ev[p], ev[p + 1]));
          acc[p] += t;
        }
      }
    } catch (...) {
      for (auto& e : ev) (void)hipEventDestroy(e);
      throw;
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
    for (int p = 0; p < 4; ++p) ms[p] = acc[p] / reps;
  });
}

extern "C" cpm_status cpm_autotune(cpm_band* b, int dtype, int nrhs, const void* u, void* v,
                                   int reps, void* hip_stream, double* ms, int* best) {
  return guard([&] {
    check_vec_args(b, dtype, nrhs, u, v);
    if (reps < 1) CPM_FAIL(CPM_E_INVALID, "reps must be >= 1");
    hipStream_t st = (hipStream_t)hip_stream;
    Tune& tn = b->tune[dtype == CPM_F64 ? 0 : 1];
    const Tune saved = tn;
    hipEvent_t e0, e1;
    CPM_HIP(hipEventCreate(&e0));
    CPM_HIP(hipEventCreate(&e1));
    double t[kTuneVariants];
    int arg = 0;
    try {
      for (int k = 0; k < kTuneVariants; ++k) {
        tn = tune_variant(k);
        if (tn.ps && b->tile_inst) {   // composites run the non-persistent gather
          t[k] = HUGE_VAL;
          continue;
        }
        auto run = [&] {
          if (dtype == CPM_F64) apply_impl<double>(b, 0.0, -1.0, nrhs, (const double*)u, (double*)v, st);
          else apply_impl<float>(b, 0.0, -1.0, nrhs, (const float*)u, (float*)v, st);
        };
        run();   // warm up
        CPM_HIP(hipEventRecord(e0, st));
        for (int r = 0; r < reps; ++r) run();
        CPM_HIP(hipEventRecord(e1, st));
        CPM_HIP(hipEventSynchronize(e1));
        float f = 0.f;
        CPM_HIP(hipEventElapsedTime(&f, e0, e1));
        t[k] = f / reps;
        if (t[k] < t[arg]) arg = k;
      }
    } catch (...) {
      tn = saved;
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    tn = tune_variant(arg);
    if (ms)
      for (int k = 0; k < kTuneVariants; ++k) ms[k] = t[k];
    if (best) *best = arg;
  });
}

extern "C" cpm_status cpm_tune_set(cpm_band* b, int dtype, int variant) {
  return guard([&] {
    if (!b) CPM_FAIL(CPM_E_INVALID, "null band");
    if (dtype != CPM_F64 && dtype != CPM_F32) CPM_FAIL(CPM_E_INVALID, "unknown dtype %d", dtype);
    if (variant < 0 || variant >= kTuneVariants)
      CPM_FAIL(CPM_E_INVALID, "launch variant %d out of range [0, %d)", variant, kTuneVariants);
    b->tune[dtype == CPM_F64 ? 0 : 1] = tune_variant(variant);
  });
}

extern "C" cpm_status cpm_apply_transpose(const cpm_band* b, double m, double n, int dtype,
                                          int nrhs, const void* w, void* z, void* hip_stream) {
  return guard([&] {
    check_vec_args(b, dtype, nrhs, w, z);
    hipStream_t st = (hipStream_t)hip_stream;
    if (dtype == CPM_F64)
      apply_transpose_impl<double>(b, m, n, nrhs, (const double*)w, (double*)z, st);
    else
      apply_transpose_impl<float>(b, m, n, nrhs, (const float*)w, (float*)z, st);
  });
}

extern "C" cpm_status cpm_rhs(const cpm_band* b, double n, int nrhs, const double* f,
                              const double* g, double* out, void* hip_stream) {
  return guard([&] {
    if (!b || !f || !out || nrhs < 1) CPM_FAIL(CPM_E_INVALID, "bad argument");
    if (b->n_c && !g) CPM_FAIL(CPM_E_INVALID, "g is required when the band has BC DOFs");
    hipStream_t st = (hipStream_t)hip_stream;
    const int64_t total = b->n * nrhs;
    hipLaunchKernelGGL(k_rhs_init, dim3(grid_for(total, 256)), dim3(256), 0, st, b->n_s, b->n_c,
                       nrhs, f, b->bc_node, out);
    CPM_LAUNCH_CHECK();
    if (g) add_dirichlet_term(b, n, g, nrhs, out, st);
  });
}

namespace cpm {
// out -= n (L - diag L) e(g) over the rows that reference BC DOFs: the
// Dirichlet part of the right-hand side (Sec. 4.3), nrhs vectors.
void add_dirichlet_term(const cpm_band* b, double n, const double* g, int nrhs, double* out,
                        hipStream_t st) {
  if (!b->n_c || !b->n_lrows) return;
  const double N2 = (double)b->N * (double)b->N;
  hipLaunchKernelGGL(k_rhs_rows, dim3(grid_for(b->n_lrows, 128)), dim3(128), 0, st, b->n_lrows,
                     2 * b->dim, b->n_s, b->n_c, nrhs, b->lrow_id, b->lcol, g, b->bc_ecoef,
                     n * N2, out);
  CPM_LAUNCH_CHECK();
}
}  // namespace cpm

extern "C" cpm_status cpm_rhs_adjoint(const cpm_band* b, double n, int nrhs, const double* lam,
                                      double* grad_f, double* grad_g, void* hip_stream) {
  return guard([&] {
    if (!b || !lam || !grad_f || nrhs < 1) CPM_FAIL(CPM_E_INVALID, "bad argument");
    hipStream_t st = (hipStream_t)hip_stream;
    hipLaunchKernelGGL(k_gradf, dim3(grid_for(b->n_s * nrhs, 256)), dim3(256), 0, st, b->n_s,
                       b->n_c, nrhs, lam, grad_f);
    CPM_LAUNCH_CHECK();
    if (b->n_c) {
      hipLaunchKernelGGL(k_gradf_bc, dim3(grid_for(b->n_c * nrhs, 256)), dim3(256), 0, st,
                         b->n_s, b->n_c, nrhs, b->bc_node, lam, grad_f);
      CPM_LAUNCH_CHECK();
    }
    if (grad_g && b->n_c) {
      CPM_HIP(hipMemsetAsync(grad_g, 0, sizeof(double) * b->n_c * nrhs, st));
      const double N2 = (double)b->N * (double)b->N;
      hipLaunchKernelGGL(k_gradg, dim3(grid_for(b->n_lrows, 128)), dim3(128), 0, st, b->n_lrows,
                         2 * b->dim, b->n_s, b->n_c, nrhs, b->lrow_id, b->lcol, lam,
                         b->bc_ecoef, -n * N2, grad_g);
      CPM_LAUNCH_CHECK();
    }
  });
}
