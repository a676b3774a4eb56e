/*
 * cpm.h - C ABI of libcpm: the closest point method (CPM) with interior
 * boundary conditions on one AMD Instinct MI355X (gfx950).
 *
 * Method: King, Su, Aanjaneya, Ruuth, Batty, "A Closest Point Method for PDEs
 * on Manifolds with Interior Boundary Conditions for Geometry Processing",
 * ACM TOG 2024 (arXiv 2305.04711).
 *
 * Conventions shared by every entry point
 *  - Grid: nodes x_k = k / N, k in Z^d, spacing h = 1/N (Sec. 3.2).
 *  - Unknowns (Sec. 4.1): n = n_s + n_c values.  PDE DOFs 0..n_s-1 are the
 *    band nodes in the library's block order (see cpm_band_export
 *    CPM_EXPORT_COORDS for their grid coordinates); BC DOFs n_s..n-1 follow,
 *    grouped by interior boundary in the order given, each group in the
 *    order of its nodes' PDE DOFs.
 *  - System (Sec. 5.4): A = m I + n [diag(L) + (L - diag L) E], with E the
 *    closest-point extension by tensor-product cubic (or quadratic, Sec. 7)
 *    Lagrange interpolation
 *    (eq. interp-stencil) with interior-boundary swaps (eq.
 *    stencil-crossing-test, eq. FD-crossing-test) and L the 2d+1-point
 *    Laplacian (eq. FD-stencil).  The affine Dirichlet part of E is moved to
 *    the right-hand side: A u = f - n (L - diag L) e(g) (see cpm_rhs).
 *  - Multi-RHS vectors are stored right-hand side by right-hand side:
 *    element (j, i) of an nrhs x len array is at [j * len + i].
 *  - Device pointers are HIP device memory of the current device; the caller
 *    owns every vector passed in.  A band owns its internal arrays and
 *    scratch vectors, taken from the cpm_allocator given to cpm_build_band,
 *    and frees them in cpm_band_free.
 *  - Every call that takes hip_stream enqueues its work on that stream
 *    (NULL = the null stream).  cpm_apply, cpm_apply_transpose, cpm_rhs and
 *    cpm_rhs_adjoint return without synchronising; cpm_build_band, the solves
 *    and cpm_band_export synchronise the stream before returning.
 *  - Errors: every call returns a cpm_status; on failure cpm_last_error()
 *    gives a message for the calling thread.  No exception crosses the ABI.
 */
#ifndef CPM_H
#define CPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CPM_OK = 0,
  CPM_E_INVALID = -1,        /* bad argument, unsupported option            */
  CPM_E_STENCIL_HOLE = -2,   /* an interpolation member is not a band node  */
  CPM_E_OOM = -3,            /* device allocation failed                    */
  CPM_E_HIP = -4,            /* a HIP runtime call failed                   */
  CPM_E_NOCONV = -5,         /* solve did not reach tol within maxit        */
  CPM_E_BREAKDOWN = -6,      /* Krylov breakdown that restarts did not cure */
  CPM_E_REACH = -7,          /* h too large for the surface's reach         */
  CPM_E_OVERLAP = -8         /* check regions of two interior boundaries meet */
} cpm_status;

/* ---- geometry (closest-point representations, App. A: analytic) ------- */
enum { CPM_SURF_CIRCLE = 1,  /* R^2: centre, R                          */
       CPM_SURF_SPHERE = 2,  /* R^3: centre, R                          */
       CPM_SURF_TORUS = 3 }; /* R^3: centre, R (core), rho (tube); axis z */

typedef struct {
  int kind;
  double center[3];
  double R;
  double rho;
} cpm_surface;

enum { CPM_IBC_POINT = 1,     /* C = {p}; orient = o_C given by the caller   */
       CPM_IBC_LATITUDE = 2,  /* sphere only: circle at height center_z + z0 */
       CPM_IBC_MERIDIAN = 3,  /* torus only: poloidal circle in the vertical
                                 plane with horizontal unit direction dir   */
       CPM_IBC_LATITUDE_ARC = 4 }; /* sphere only: the open arc of the
                                 LATITUDE circle running counter-clockwise
                                 from the horizontal unit direction
                                 (arc[0], arc[1]) to (arc[2], arc[3]) (Sec.
                                 4.4: no BC DOF and no stencil change where
                                 cp_C is an endpoint)                       */

/* Condition imposed on one side of an interior boundary (Sec. 4.3).  Each
 * side carries its own (Sec. 4.2: two-sided and mixed IBCs).  The sides are
 * told apart by the orientation o_C: side +1 is where (cp_S - cp_C) . o_C >= 0
 * (POINT: the caller's orient; LATITUDE: north; MERIDIAN: the plane normal
 * (-ey, ex, 0)). */
enum { CPM_BC_DIRICHLET = 0,  /* u = g on C: first order extends g, second
                                 order 2 g - u at the mirror point cpbar_C  */
       CPM_BC_NEUMANN = 1 };  /* zero conormal derivative on C: the BC DOF
                                 interpolates u at cp_C (first order) or at
                                 cpbar_C = cp_S(2 cp_C - x) (second order);
                                 not defined for a point C                   */

typedef struct {
  int kind;
  double p[3];       /* POINT: the point (on S)                               */
  double orient[3];  /* POINT: o_C, the side a closest point lying on C
                        (within tau of it) is assigned to (Sec. 4.2)          */
  double z0;         /* LATITUDE                                              */
  double dir[2];     /* MERIDIAN: (ex, ey), a unit vector                     */
  int bc[2];         /* CPM_BC_* of side +1 and of side -1; zero-initialised
                        = Dirichlet on both sides                            */
  double arc[4];     /* LATITUDE_ARC: start and end directions (unit)         */
} cpm_ibc;

typedef struct {
  int N;               /* h = 1/N                                             */
  int p;               /* interpolation degree: 3 (cubic) or 2 (quadratic,
                          nearest-node stencils, Sec. 7)                     */
  int order;           /* IBC order (Dirichlet and Neumann): 1 or 2 (Sec. 4.3) */
  int check_reach;     /* 1: reject h above the reach bound (Sec. 8 grid
                          resolution in practice)                           */
  double r_band;       /* 0 = eq. (bandwidth) with q = 1                      */
  double tau_factor;   /* 0 = 0.1: on-C tolerance tau = tau_factor h^2 (Sec. 4.2) */
  double check_factor; /* 0 = 2: check region ||x - cp_C(x)|| < check_factor r (Sec. 4.6) */
  int band;            /* CPM_BAND_TUBE (0): every node within r (eq.
                          bandwidth); CPM_BAND_STENCIL_SET (1): only the nodes
                          of the tube's DOFs that some interpolation stencil
                          uses and the FD neighbours of their rows (Sec. 5.1
                          cites this construction); on the stencil-referenced
                          DOFs the system, hence the solution, is the tube's  */
} cpm_grid;

enum { CPM_BAND_TUBE = 0, CPM_BAND_STENCIL_SET = 1 };

typedef struct cpm_band cpm_band;

/* Device memory provider.  The paper's solver (Sec. 5.4) holds the band's
 * stencil data and the Krylov vectors in memory it allocates itself; here
 * the caller can own that memory instead (for example a framework's caching
 * allocator, so that one pool serves the caller's tensors and the band).
 *   alloc(bytes, hip_stream, ctx): device memory of at least `bytes` bytes on
 *     the current device, usable in stream order on hip_stream, or NULL on
 *     failure (the call then returns CPM_E_OOM).
 *   free(ptr, bytes, hip_stream, ctx): return a block alloc gave, with the
 *     size it was asked for.
 * Both get the stream given when the band (or batch) was created.  The
 * library synchronises that stream after each alloc, before it uses the
 * block on other streams, and synchronises the device before it frees a
 * block that kernels may have used (a scratch vector that grows, and
 * everything at cpm_band_free / cpm_batch_free).  The callbacks are called
 * from the thread making the library call and must not call back into the
 * library.  The struct is copied; ctx must outlive the band. */
typedef struct {
  void* (*alloc)(size_t bytes, void* hip_stream, void* ctx);
  void (*free)(void* ptr, size_t bytes, void* hip_stream, void* ctx);
  void* ctx;
} cpm_allocator;

typedef struct {
  int dim, N, n_ibc, order;
  int64_t n_s, n_c, n;          /* PDE, BC and total DOFs                     */
  int64_t n_blocks;             /* occupied 4x4x4 (8x8 in 2-D) blocks         */
  int64_t n_tiles;              /* gather tiles (occupied stencil-base blocks) */
  int64_t n_erows, n_lrows;     /* rows with explicit E / L stencils           */
  int64_t on_c_nodes;           /* nodes whose cp_S lies within tau of C      */
  int64_t no_bc_dof_swaps;      /* opposite-side members with no BC DOF       */
  double h, r_band, tau;
  size_t device_bytes;          /* bytes of the band's arrays on the device   */
  size_t scratch_bytes;         /* bytes of its scratch vectors at this time
                                   (grown by applies and solves)             */
} cpm_band_info;

/* Build the band Omega(S) (eq. bandwidth, Alg. 1 semantics: every node within
 * r of S), Omega(C), the check region and side vectors for each interior
 * boundary (Sec. 4.1, 4.2, 4.6), the interpolation and FD stencils with their
 * swaps and the BC-DOF rows (Sec. 4.3).  Membership and stencil decisions are
 * taken in FP64 in a fixed evaluation order.
 *   ibcs may be NULL when n_ibc == 0.  allocator: every device allocation of
 *   the band goes through it (its arrays, the build's temporaries, and the
 *   scratch vectors later calls grow on demand); NULL = hipMalloc / hipFree.
 *   On success *out owns that memory until cpm_band_free.
 *   Errors: CPM_E_INVALID (N <= 0, p not 2 or 3, unknown kind, IBC kind that
 *   does not fit the surface), CPM_E_REACH, CPM_E_STENCIL_HOLE (message gives
 *   the count), CPM_E_OVERLAP, CPM_E_OOM, CPM_E_HIP. */
cpm_status cpm_build_band(const cpm_surface* surface, const cpm_ibc* ibcs,
                          int n_ibc, const cpm_grid* grid,
                          const cpm_allocator* allocator, void* hip_stream,
                          cpm_band** out);

void cpm_band_free(cpm_band* band);

cpm_status cpm_band_query(const cpm_band* band, cpm_band_info* out);

/* Copy band data to host memory in DOF order (for parity checks and for
 * evaluating data at closest points, Sec. 5.2).  bytes must equal the size
 * stated for `what`; otherwise CPM_E_INVALID. */
enum {
  CPM_EXPORT_COORDS = 1,   /* int32 [n_s][d]  grid coordinates k             */
  CPM_EXPORT_CP = 2,       /* double [n_s][d] stored cp_S(x_k)               */
  CPM_EXPORT_BC_NODE = 3,  /* int32 [n_c]     PDE DOF of each BC DOF's node  */
  CPM_EXPORT_BC_CPC = 4,   /* double [n_c][d] cp_C at that node              */
  CPM_EXPORT_BC_SIDE = 5,  /* int32 [n_c]     own side (+1/-1, sign v.o_C)   */
  CPM_EXPORT_BC_CURVE = 6, /* int32 [n_c]     index of the interior boundary */
  CPM_EXPORT_ECOLS = 7,    /* int32 [n][4^d]  E columns after swaps, member
                              o = (o%4, o/4%4, o/16) from the base; -1 none */
  CPM_EXPORT_LCOLS = 8,    /* int32 [n][2d]   L off-diagonal columns after
                              swaps in order -x,+x,-y,+y,-z,+z; -1 dropped  */
  CPM_EXPORT_BASE = 9      /* int32 [n][d]    interpolation stencil base
                              (BC rows: of the mirror point; 0 if none)     */
};
cpm_status cpm_band_export(const cpm_band* band, int what, void* host_dst,
                           size_t bytes);

enum { CPM_F64 = 0, CPM_F32 = 1 };

/* v = A u for the linear part of A (Sec. 5.4, four-step product: a = E u,
 * b = (L - diag L) a, then v = m u + n diag(L) u + n b), nrhs right-hand
 * sides.  dtype CPM_F64: u, v are double; CPM_F32: u, v are float and the
 * stored interpolation fractions are read in FP32, but weights, products,
 * sums and the intermediate a are FP64 for both dtypes (the Laplacian
 * differences neighbouring values of a and scales them by 1/h^2, which would
 * amplify an FP32 rounding of a by 1/h^2); the result is rounded to the
 * dtype once.  u and v are device arrays [nrhs][n] and must not alias.
 * Scratch: an FP64 vector of n * nrhs held by the band (allocated on first
 * use and reused). */
cpm_status cpm_apply(const cpm_band* band, double m, double n, int dtype,
                     int nrhs, const void* u, void* v, void* hip_stream);

/* cpm_apply without device allocation, for callers that cannot allocate:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, result (bit for bit) and precision as
 * cpm_apply, through the same kernels.  The FP64 intermediate a = E u lives
 * in a static device array of the library (32 MiB on each GPU it runs on,
 * held until the process ends) instead of the band's scratch, so
 * n * nrhs <= 4194304 is required: larger calls return CPM_E_INVALID with
 * nothing enqueued.  The array's address is looked up on the first call on
 * each device.  Every call on one GPU shares the array: calls that may
 * overlap on one GPU (on different streams, or from several threads) race
 * on it and must be serialised by the caller. */
cpm_status cpm_apply_noalloc(const cpm_band* band, double m, double n, int dtype,
                             int nrhs, const void* u, void* v, void* hip_stream);

/* z = A^T w = m w + n diag(L) w + n E^T ((L - diag L)^T w): the transpose of
 * cpm_apply (derived from Sec. 5.4).  Every sum has a fixed order (per-tile
 * LDS cubes added class by class; explicit rows through pull lists), so the
 * result is the same bit for bit on every call.  Arguments and precision as
 * for cpm_apply (FP64 intermediates (L - diag L)^T w and E^T of it for both
 * dtypes); CPM_E_INVALID also for a band without a transpose schedule. */
cpm_status cpm_apply_transpose(const cpm_band* band, double m, double n,
                               int dtype, int nrhs, const void* w, void* z,
                               void* hip_stream);

/* b = P f - n (L - diag L) e(g): f [nrhs][n_s] is the closest-point
 * extension of the source (Sec. 5.2), copied to each BC DOF from the PDE DOF
 * of its node; g [nrhs][n_c] holds the Dirichlet value each BC DOF enforces,
 * e(g) = g (first order) or 2 g (second order) on BC DOFs (Sec. 4.3).
 * g may be NULL when n_c == 0.  Device pointers, double; b is [nrhs][n]. */
cpm_status cpm_rhs(const cpm_band* band, double n, int nrhs, const double* f,
                   const double* g, double* b, void* hip_stream);

/* Gradients of a scalar loss through b(f, g) given lambda = A^-T dl/du:
 * grad_f = P^T lambda [nrhs][n_s], grad_g = -n c (L - diag L)^T lambda on
 * the BC DOFs [nrhs][n_c] (c = 1 or 2 as above).  grad_g may be NULL. */
cpm_status cpm_rhs_adjoint(const cpm_band* band, double n, int nrhs,
                           const double* lambda, double* grad_f,
                           double* grad_g, void* hip_stream);

enum { CPM_SOLVE_MIXED = 0,  /* FP32 BiCGSTAB (FP32 vectors, the CPM_F32
                                apply, FP64 partial solution) with FP64
                                reliable updates                          */
       CPM_SOLVE_F64 = 1,    /* plain FP64 BiCGSTAB                        */
       CPM_SOLVE_GMRES = 2 };/* FP64 restarted GMRES(restart), classical
                                Gram-Schmidt with one re-orthogonalisation  */

typedef struct {
  double m, n;        /* A = m I + n M                                       */
  double tol;         /* stop when ||b - A x||_2 <= tol ||b||_2 (FP64)       */
  int mode;           /* CPM_SOLVE_MIXED or CPM_SOLVE_F64                    */
  int maxit;          /* cap on Krylov iterations in total (0 = 20000)       */
  double inner_tol;   /* mixed: reliable-update factor delta (0 = 0.1): once
                         the FP32 recursive residual has dropped by delta
                         since the last update, the partial solution is
                         added into x in FP64 and the FP32 recurrence
                         restarts from the FP64 true residual               */
  int check_every;    /* iterations between convergence read-backs (0 = 16)  */
  int use_graph;      /* 1: replay the check_every iterations as a hipGraph  */
  double gauge;       /* >0: solve (A + gauge 1 w^T) x = b, w = 1/n_s on PDE
                         DOFs (closed-surface Poisson); 0 = off              */
  int restart;        /* GMRES restart length (0 = 50, at most 200)          */
} cpm_solve_opts;

typedef struct {
  int converged;
  int outer_iters;    /* FP64 residual evaluations (mixed: reliable updates) */
  int krylov_iters;   /* BiCGSTAB iterations in total                       */
  int restarts;       /* breakdown restarts                                 */
  int fallback_f64;   /* mixed: updates stalled, finished in plain FP64      */
  double relres;      /* final true FP64 relative residual (max over RHS)   */
  double time_ms;     /* wall time of the call                              */
} cpm_solve_stats;

/* Solve A x = b (Sec. 5.4) for nrhs right-hand sides; b and x are device
 * double arrays [nrhs][n]; x holds the initial guess on entry (warm start)
 * and the solution on return.  On CPM_E_NOCONV x holds the last iterate and
 * stats are filled.  stats may be NULL. */
cpm_status cpm_solve(const cpm_band* band, const cpm_solve_opts* opts,
                     int nrhs, const double* b, double* x,
                     cpm_solve_stats* stats, void* hip_stream);

/* Solve A^T lambda = rhs (same options and conventions as cpm_solve). */
cpm_status cpm_solve_adjoint(const cpm_band* band, const cpm_solve_opts* opts,
                             int nrhs, const double* rhs, double* lambda,
                             cpm_solve_stats* stats, void* hip_stream);

/* Crank-Nicolson time stepping of u_t = Delta_S u (the heat test of Sec.
 * 6.2; trapezoidal rule) on the band's system with its interior boundaries:
 *   (I - dt/2 M) u^{k+1} = (I + dt/2 M) u^k + dt/2 (L - D)(e(g^k) + e(g^{k+1}))
 * for k = 0 .. nsteps-1, with M = diag L + (L - diag L) E.  u: device double
 * [n], u^0 on entry and u^nsteps on return (updated in place step by step).
 * g: device double [nsteps + 1][n_c], the Dirichlet data at t_k = k dt (only
 * Dirichlet BC DOFs read it; NULL when there are none).  opts: mode, tol,
 * maxit, check_every, use_graph and inner_tol as for cpm_solve (m, n are
 * set by the scheme; the gauge must be 0); each step is warm-started from
 * u^k.  stats (may be NULL): iterations summed over the steps, worst relative
 * residual.  A step that does not converge stops the run with CPM_E_NOCONV
 * (u then holds that step's last iterate). */
cpm_status cpm_heat_cn(const cpm_band* band, double dt, int nsteps,
                       const double* g, double* u, const cpm_solve_opts* opts,
                       cpm_solve_stats* stats, void* hip_stream);

/* Measurement: run cpm_apply `reps` times on hip_stream with HIP events
 * around each of its four phases and return the mean milliseconds per call in
 * ms[4]: [0] tile gather (a = E u for rows without swaps), [1] explicit
 * interpolation rows, [2] block Laplacian pass, [3] explicit FD rows.
 * Synchronises the stream.  Arguments as for cpm_apply. */
cpm_status cpm_apply_profile(const cpm_band* band, double m, double n, int dtype,
                             int nrhs, const void* u, void* v, int reps,
                             void* hip_stream, double* ms);

/* ---- batched solves (several bands, uneven sizes, nrhs each) ----------
 * A batch concatenates the bands' device data once (DOFs of band i at
 * [offsets[i], offsets[i+1]) of a batch vector of length total) so that one
 * launch per kernel applies every instance; band i uses A_i = m[i] I + n[i] M_i.
 * Batch vectors are [nrhs][total].  The bands must stay alive while the batch
 * is used; they must all have the same dimension.  The batch's own device
 * memory (the composite band, its scratch and the solver's segment tables)
 * comes from allocator as for cpm_build_band (NULL = hipMalloc / hipFree). */
typedef struct cpm_batch cpm_batch;
cpm_status cpm_batch_create(cpm_band* const* bands, int nbands, const double* m,
                            const double* n, int nrhs,
                            const cpm_allocator* allocator, void* hip_stream,
                            cpm_batch** out);
void cpm_batch_free(cpm_batch* batch);
/* offsets: nbands + 1 entries; offsets[nbands] = total */
cpm_status cpm_batch_offsets(const cpm_batch* batch, int64_t* offsets);
/* v = A u for every instance and right-hand side (dtype CPM_F64 / CPM_F32) */
cpm_status cpm_batch_apply(const cpm_batch* batch, int dtype, const void* u,
                           void* v, void* hip_stream);
/* Autotune the batch's apply as cpm_autotune does for one band (its timing
 * vectors are scratch of the batch, kept for later calls). */
cpm_status cpm_batch_autotune(cpm_batch* batch, int dtype, int reps,
                              void* hip_stream, double* ms, int* best);
/* Solve every system (instance, right-hand side) with its own BiCGSTAB
 * scalars and convergence flag; opts->m, n and gauge are not used (the batch
 * holds m, n per instance; the gauge is not supported).  Mixed mode refines
 * in FP64 per system with FP32 steps (FP32 recurrence, the CPM_F32 apply,
 * FP64 partial solution) to the relative tolerance inner_tol (0 = 1e-2) and
 * finishes in FP64 any system whose FP64 residual did not halve over a
 * step.  rhs and x are device [nrhs][total] double; x holds x0 on entry.
 * stats (may be NULL): nrhs * nbands entries, system s = r * nbands + i. */
cpm_status cpm_batch_solve(cpm_batch* batch, const cpm_solve_opts* opts,
                           const double* rhs, double* x, cpm_solve_stats* stats,
                           void* hip_stream);

/* Autotuner: time every launch variant of cpm_apply for this band, dtype and
 * nrhs with HIP events, `reps` calls each, and keep the fastest for later
 * calls with this dtype.  Variant k = 8 lap + 2 mode + pad (0 <= k < 32):
 * pad is the LDS line padding of the staged cube (0: 1 element, 1: 4
 * elements); mode 0 visits tiles and blocks in block order, mode 1 gives each
 * XCD a contiguous range of them, mode 2 runs the tile gather as persistent
 * wavefronts over such ranges that request the next tile's metadata early,
 * mode 3 also its staged values (modes 2 and 3 are for bands only: a batch's
 * composite skips them and reports HUGE_VAL); lap 0 gathers every FD
 * neighbour of the Laplacian pass from memory, lap 1 exchanges in-block
 * neighbours between lanes, lap 2 does the same in persistent wavefronts
 * that request the next block's data while finishing the current one (one
 * right-hand side; with several the pass runs as lap 1), lap 3 takes two
 * blocks per wavefront with their metadata in scalar registers and exchanges
 * in-block neighbours with row moves and lane permutes.  u and v are
 * scratch device arrays [nrhs][n] of that dtype.  ms (may be NULL) receives
 * the 32 mean times per call; *best (may be NULL) the chosen variant.
 * Synchronises the stream. */
cpm_status cpm_autotune(cpm_band* band, int dtype, int nrhs, const void* u,
                        void* v, int reps, void* hip_stream, double* ms,
                        int* best);

/* Select launch variant k (numbered as by cpm_autotune, 0 <= k < 32) for
 * later calls on this band with this dtype, without timing anything; every
 * variant computes each output entry with the same arithmetic.  Returns
 * CPM_E_INVALID for a k out of range.  Touches no device memory. */
cpm_status cpm_tune_set(cpm_band* band, int dtype, int variant);

const char* cpm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* CPM_H */
