"""Python binding of libcpm with the same entry points as the C ABI
(include/cpm.h): build_band, apply (apply_cpm), apply_transpose, rhs,
rhs_adjoint, solve, solve_adjoint, and CPMSolve, a torch.autograd.Function
whose backward is the hand-written adjoint.

PyTorch provides device memory and streams only; every step of the method
runs in libcpm's HIP kernels.  Vectors are torch tensors on the current HIP
device, shaped (n,) or (nrhs, n).
"""

import atexit
import ctypes as C
import weakref

import numpy as np
import torch

from . import capi


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr())


# ------------------------------------------------------------------ memory
# The torch caching allocator as the library's cpm_allocator: the band's
# arrays and scratch vectors come from the same pool as the caller's tensors
# (torch.cuda.memory_allocated counts them).  The callbacks run on the thread
# that calls into the library, which holds no GIL during the call; ctypes
# takes the GIL for them.
def _torch_alloc(nbytes, stream, ctx):
    try:
        return int(torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0)))
    except Exception:   # out of memory: the library reports CPM_E_OOM
        return 0


def _torch_free(ptr, nbytes, stream, ctx):
    try:
        torch.cuda.caching_allocator_delete(int(ptr))
    except Exception:
        pass


_TORCH_ALLOCATOR = capi.Allocator(capi.ALLOC_FN(_torch_alloc), capi.FREE_FN(_torch_free), None)

# Bands and batches still open at interpreter exit are freed while the
# callbacks above (and torch) are still alive.
_LIVE = weakref.WeakSet()


@atexit.register
def _close_all():
    for obj in list(_LIVE):
        try:
            obj.close()
        except Exception:
            pass


def _allocator(kind):
    """kind "torch" (default): the torch caching allocator; None: hipMalloc."""
    if kind == "torch":
        return C.byref(_TORCH_ALLOCATOR)
    if kind is None:
        return None
    raise ValueError("allocator is 'torch' or None")


# ------------------------------------------------------------------ geometry
def circle(R=1.0, center=(0.0, 0.0)):
    return capi.Surface(capi.SURF_CIRCLE, (C.c_double * 3)(center[0], center[1], 0.0), R, 0.0)


def sphere(R=1.0, center=(0.0, 0.0, 0.0)):
    return capi.Surface(capi.SURF_SPHERE, (C.c_double * 3)(*center), R, 0.0)


def torus(R=1.0, rho=0.4, center=(0.0, 0.0, 0.0)):
    return capi.Surface(capi.SURF_TORUS, (C.c_double * 3)(*center), R, rho)


_BC = {"dirichlet": capi.BC_DIRICHLET, "neumann": capi.BC_NEUMANN}


def _bc(bc):
    """(condition of side +1, condition of side -1), "dirichlet" or "neumann"."""
    if isinstance(bc, str):
        bc = (bc, bc)
    return (C.c_int * 2)(_BC[bc[0]], _BC[bc[1]])


def point_ibc(p, orient):
    p = list(p) + [0.0] * (3 - len(p))
    o = list(orient) + [0.0] * (3 - len(orient))
    return capi.IBC(capi.IBC_POINT, (C.c_double * 3)(*p), (C.c_double * 3)(*o), 0.0,
                    (C.c_double * 2)(0.0, 0.0), _bc("dirichlet"))


def latitude_ibc(z0, bc="dirichlet"):
    return capi.IBC(capi.IBC_LATITUDE, (C.c_double * 3)(), (C.c_double * 3)(), z0,
                    (C.c_double * 2)(0.0, 0.0), _bc(bc))


def latitude_arc_ibc(z0, a, b, bc="dirichlet"):
    """Open arc of the latitude circle from unit direction a to unit direction
    b, counter-clockwise (Sec. 4.4)."""
    ib = capi.IBC(capi.IBC_LATITUDE_ARC, (C.c_double * 3)(), (C.c_double * 3)(), z0,
                  (C.c_double * 2)(0.0, 0.0), _bc(bc))
    ib.arc[0], ib.arc[1], ib.arc[2], ib.arc[3] = float(a[0]), float(a[1]), float(b[0]), float(b[1])
    return ib


def meridian_ibc(ex, ey, bc="dirichlet"):
    return capi.IBC(capi.IBC_MERIDIAN, (C.c_double * 3)(), (C.c_double * 3)(), 0.0,
                    (C.c_double * 2)(ex, ey), _bc(bc))


# ------------------------------------------------------------------ band
class Band:
    """cpm_build_band: the narrow band, interior-boundary DOFs and stencils
    for one surface and grid (h = 1/N).  band: "tube" (eq. bandwidth) or
    "stencil_set" (only the nodes interpolation and FD stencils need)."""

    def __init__(self, surface, ibcs=(), N=64, order=2, r_band=0.0, tau_factor=0.0,
                 check_factor=0.0, check_reach=False, p=3, band="tube", allocator="torch"):
        kinds = {"tube": capi.BAND_TUBE, "stencil_set": capi.BAND_STENCIL_SET}
        if band not in kinds:
            raise ValueError("band is 'tube' or 'stencil_set'")
        lib = capi.load()
        self._lib = lib
        self.handle = None
        arr = (capi.IBC * max(1, len(ibcs)))(*ibcs) if ibcs else None
        grid = capi.Grid(int(N), int(p), int(order), int(bool(check_reach)), float(r_band),
                         float(tau_factor), float(check_factor), kinds[band])
        out = C.c_void_p()
        capi.check(lib.cpm_build_band(C.byref(surface), arr, len(ibcs), C.byref(grid),
                                      _allocator(allocator), _stream(), C.byref(out)))
        self.handle = out
        _LIVE.add(self)
        info = capi.BandInfo()
        capi.check(lib.cpm_band_query(self.handle, C.byref(info)))
        self.info = {k: getattr(info, k) for k, _ in capi.BandInfo._fields_}
        self.dim = info.dim
        self.N = info.N
        self.n_s, self.n_c, self.n = info.n_s, info.n_c, info.n

    def close(self):
        if self.handle is not None and self.handle.value:
            self._lib.cpm_band_free(self.handle)
        self.handle = None

    def memory(self):
        """(array bytes, scratch bytes) the band holds on the device now."""
        info = capi.BandInfo()
        capi.check(self._lib.cpm_band_query(self.handle, C.byref(info)))
        return info.device_bytes, info.scratch_bytes

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _export(self, what, dtype, shape):
        out = np.empty(shape, dtype=dtype)
        if out.size:
            capi.check(self._lib.cpm_band_export(self.handle, what,
                                                 out.ctypes.data_as(C.c_void_p), out.nbytes))
        return out

    def coords(self):
        return self._export(capi.EXPORT_COORDS, np.int32, (self.n_s, self.dim))

    def cp(self):
        return self._export(capi.EXPORT_CP, np.float64, (self.n_s, self.dim))

    def bc_node(self):
        return self._export(capi.EXPORT_BC_NODE, np.int32, (self.n_c,))

    def bc_cpc(self):
        return self._export(capi.EXPORT_BC_CPC, np.float64, (self.n_c, self.dim))

    def bc_side(self):
        return self._export(capi.EXPORT_BC_SIDE, np.int32, (self.n_c,))

    def bc_curve(self):
        return self._export(capi.EXPORT_BC_CURVE, np.int32, (self.n_c,))

    def ecols(self):
        return self._export(capi.EXPORT_ECOLS, np.int32, (self.n, 4 ** self.dim))

    def lcols(self):
        return self._export(capi.EXPORT_LCOLS, np.int32, (self.n, 2 * self.dim))

    def bases(self):
        return self._export(capi.EXPORT_BASE, np.int32, (self.n, self.dim))


def build_band(surface, ibcs=(), N=64, **kw):
    return Band(surface, ibcs, N, **kw)


# ------------------------------------------------------------------ operators
def _dtype_code(t):
    if t.dtype == torch.float64:
        return capi.F64
    if t.dtype == torch.float32:
        return capi.F32
    raise TypeError("vectors must be float64 or float32")


def _check_vec(band, t, length):
    if not t.is_cuda:
        raise ValueError("vectors must be on the GPU (no CPU path)")
    if not t.is_contiguous():
        raise ValueError("vectors must be contiguous")
    if t.dim() not in (1, 2):
        raise ValueError("vectors are 1-D (n,) or 2-D (nrhs, n)")
    if t.shape[-1] != length:
        raise ValueError("last dimension must be %d (got %d)" % (length, t.shape[-1]))
    return 1 if t.dim() == 1 else t.shape[0]


def _check_f64(t, what):
    if t.dtype != torch.float64:
        raise TypeError("%s must be float64" % what)


def _check_like(x0, b):
    """A warm start has the right-hand sides' shape, dtype and device."""
    if (not x0.is_cuda or x0.dtype != b.dtype or tuple(x0.shape) != tuple(b.shape)
            or x0.device != b.device):
        raise ValueError("x0 must be a %s device tensor of shape %s"
                         % (b.dtype, tuple(b.shape)))


def apply(band, u, m, n):
    """apply_cpm: v = A u, A = m I + n [diag L + (L - diag L) E]."""
    nrhs = _check_vec(band, u, band.n)
    v = torch.empty_like(u)
    capi.check(band._lib.cpm_apply(band.handle, float(m), float(n), _dtype_code(u), nrhs,
                                   _ptr(u), _ptr(v), _stream()))
    return v


apply_cpm = apply


def apply_profile(band, u, m, n, reps=20):
    """Mean milliseconds per phase of cpm_apply over `reps` calls, timed with
    HIP events on the launch stream: (tile gather, explicit E rows, block
    Laplacian, explicit L rows)."""
    nrhs = _check_vec(band, u, band.n)
    v = torch.empty_like(u)
    ms = (C.c_double * 4)()
    capi.check(band._lib.cpm_apply_profile(band.handle, float(m), float(n), _dtype_code(u), nrhs,
                                           _ptr(u), _ptr(v), int(reps), _stream(), ms))
    return list(ms), v


def autotune(band, dtype=torch.float64, nrhs=1, reps=10):
    """Pick the fastest apply launch variant for this band and dtype (kept in
    the band).  Returns (times_ms[capi.TUNE_VARIANTS], best): variant
    k = 8 lap + 2 mode + pad (mode 0 block order, 1 XCD-aware order, 2
    persistent XCD-aware tile gather, 3 persistent and pipelined; lap 0, 1, 2
    the three forms of the Laplacian pass)."""
    shape = (band.n,) if nrhs == 1 else (nrhs, band.n)
    u = torch.randn(shape, dtype=dtype, device="cuda")
    v = torch.empty_like(u)
    ms = (C.c_double * capi.TUNE_VARIANTS)()
    best = C.c_int()
    capi.check(band._lib.cpm_autotune(band.handle, _dtype_code(u), nrhs, _ptr(u), _ptr(v),
                                      int(reps), _stream(), ms, C.byref(best)))
    return list(ms), best.value


def tune_set(band, dtype, variant):
    """Select launch variant `variant` (numbered as by autotune) for this band
    and dtype without timing."""
    code = capi.F64 if dtype == torch.float64 else capi.F32
    capi.check(band._lib.cpm_tune_set(band.handle, code, int(variant)))


def apply_transpose(band, w, m, n):
    nrhs = _check_vec(band, w, band.n)
    z = torch.empty_like(w)
    capi.check(band._lib.cpm_apply_transpose(band.handle, float(m), float(n), _dtype_code(w),
                                             nrhs, _ptr(w), _ptr(z), _stream()))
    return z


def rhs(band, f, g, n):
    """b = P f - n (L - diag L) e(g); f (.., n_s), g (.., n_c) float64."""
    nrhs = _check_vec(band, f, band.n_s)
    _check_f64(f, "f")
    shape = (band.n,) if f.dim() == 1 else (nrhs, band.n)
    b = torch.empty(shape, dtype=torch.float64, device=f.device)
    gp = None
    if band.n_c:
        if g is None:
            raise ValueError("g is required when the band has BC DOFs")
        _check_vec(band, g, band.n_c)
        _check_f64(g, "g")
        if tuple(g.shape[:-1]) != tuple(f.shape[:-1]):
            raise ValueError("g must hold one row per right-hand side of f")
        gp = _ptr(g)
    capi.check(band._lib.cpm_rhs(band.handle, float(n), nrhs, _ptr(f), gp, _ptr(b), _stream()))
    return b


def rhs_adjoint(band, lam, n):
    nrhs = _check_vec(band, lam, band.n)
    _check_f64(lam, "lambda")
    lead = () if lam.dim() == 1 else (nrhs,)
    gf = torch.empty(lead + (band.n_s,), dtype=torch.float64, device=lam.device)
    gg = torch.zeros(lead + (band.n_c,), dtype=torch.float64, device=lam.device)
    capi.check(band._lib.cpm_rhs_adjoint(band.handle, float(n), nrhs, _ptr(lam), _ptr(gf),
                                         _ptr(gg) if band.n_c else None, _stream()))
    return gf, gg


def _opts(m, n, tol, mode, maxit, inner_tol, check_every, use_graph, gauge, restart=0):
    code = {"mixed": capi.SOLVE_MIXED, "f64": capi.SOLVE_F64, "gmres": capi.SOLVE_GMRES}[mode]
    return capi.SolveOpts(float(m), float(n), float(tol), code, int(maxit), float(inner_tol),
                          int(check_every), int(bool(use_graph)), float(gauge), int(restart))


def _solve(fn, band, b, m, n, tol, mode, x0, maxit, inner_tol, check_every, use_graph, gauge,
           raise_noconv, restart=0):
    nrhs = _check_vec(band, b, band.n)
    if b.dtype != torch.float64:
        raise TypeError("right-hand sides are float64")
    if x0 is not None:
        _check_like(x0, b)
    x = torch.zeros_like(b) if x0 is None else x0.clone().contiguous()
    st = capi.SolveStats()
    o = _opts(m, n, tol, mode, maxit, inner_tol, check_every, use_graph, gauge, restart)
    status = fn(band.handle, C.byref(o), nrhs, _ptr(b), _ptr(x), C.byref(st), _stream())
    stats = {k: getattr(st, k) for k, _ in capi.SolveStats._fields_}
    if status == capi.E_NOCONV and not raise_noconv:
        return x, stats
    capi.check(status)
    return x, stats


def heat_cn(band, u0, dt, nsteps, g=None, tol=1e-10, mode="f64", maxit=0, check_every=0,
            use_graph=True, raise_noconv=True):
    """cpm_heat_cn: nsteps Crank-Nicolson steps of u_t = Delta_S u from u0
    (float64, length n); g: float64 (nsteps + 1, n_c) Dirichlet data at the
    step times, or None.  Returns (u, stats)."""
    if _check_vec(band, u0, band.n) != 1 or u0.dim() != 1:
        raise ValueError("the state is one vector of length n")
    if u0.dtype != torch.float64:
        raise TypeError("the state is float64")
    u = u0.clone().contiguous()
    gp = None
    if g is not None:
        if g.dtype != torch.float64 or not g.is_cuda or tuple(g.shape) != (nsteps + 1, band.n_c):
            raise ValueError("g must be a float64 device tensor of shape (nsteps + 1, n_c)")
        g = g.contiguous()
        gp = _ptr(g)
    st = capi.SolveStats()
    o = _opts(1.0, -0.5 * dt, tol, mode, maxit, 0.0, check_every, use_graph, 0.0)
    status = band._lib.cpm_heat_cn(band.handle, float(dt), int(nsteps), gp, _ptr(u), C.byref(o),
                                   C.byref(st), _stream())
    stats = {k: getattr(st, k) for k, _ in capi.SolveStats._fields_}
    if status == capi.E_NOCONV and not raise_noconv:
        return u, stats
    capi.check(status)
    return u, stats


def solve(band, b, m, n, tol=1e-8, mode="mixed", x0=None, maxit=0, inner_tol=0.0,
          check_every=0, use_graph=True, gauge=0.0, raise_noconv=True, restart=0):
    """Solve A x = b.  mode "mixed": FP32 BiCGSTAB with FP64 reliable updates
    (inner_tol = update factor delta, 0 = 0.1); "f64":
    plain FP64 BiCGSTAB; "gmres": FP64 GMRES(restart).  Returns (x, stats)."""
    return _solve(band._lib.cpm_solve, band, b, m, n, tol, mode, x0, maxit, inner_tol,
                  check_every, use_graph, gauge, raise_noconv, restart)


def solve_adjoint(band, rhs_, m, n, tol=1e-8, mode="mixed", x0=None, maxit=0, inner_tol=0.0,
                  check_every=0, use_graph=True, raise_noconv=True, restart=0):
    """Solve A^T lam = rhs_ (the adjoint system), modes as for solve."""
    return _solve(band._lib.cpm_solve_adjoint, band, rhs_, m, n, tol, mode, x0, maxit,
                  inner_tol, check_every, use_graph, 0.0, raise_noconv, restart)


def _check_attained(stats, tol, what):
    """Raise unless the solve reached its tolerance.  In FP64 the true
    residual of an iterate cannot be driven (or even measured) below about
    eps64 ||A|| ||x|| / ||b||, eps64 kappa for smooth solutions (a few 1e-11
    at h = 1/128 on the test surfaces): tolerances near that floor fail here
    rather than being accepted silently."""
    if not (stats["relres"] <= tol):
        raise capi.CPMError(capi.E_NOCONV, "%s reached relative residual %.3g, above tol %.3g "
                            "(%d iterations)" % (what, stats["relres"], tol,
                                                 stats["krylov_iters"]))


class CPMSolve(torch.autograd.Function):
    """u = A^-1 b(f, g) with gradients with respect to f (n_s) and the interior
    Dirichlet values g (n_c) from the adjoint solve A^T lam = dl/du.  Both
    solves must reach tol (CPMError otherwise).  stats (optional dict)
    receives the solver statistics under "forward" and, after backward,
    "backward"."""

    @staticmethod
    def forward(ctx, f, g, band, m, n, tol=1e-10, mode="mixed", stats=None):
        b = rhs(band, f.detach().contiguous(), g.detach().contiguous() if band.n_c else None, n)
        u, st = solve(band, b, m, n, tol=tol, mode=mode, raise_noconv=False)
        if stats is not None:
            stats["forward"] = st
        _check_attained(st, tol, "forward solve")
        ctx.band, ctx.m, ctx.n, ctx.tol, ctx.mode, ctx.stats = band, m, n, tol, mode, stats
        return u

    @staticmethod
    def backward(ctx, grad_u):
        band = ctx.band
        lam, st = solve_adjoint(band, grad_u.contiguous().to(torch.float64), ctx.m, ctx.n,
                                tol=ctx.tol, mode=ctx.mode, raise_noconv=False)
        if ctx.stats is not None:
            ctx.stats["backward"] = st
        _check_attained(st, ctx.tol, "adjoint solve")
        gf, gg = rhs_adjoint(band, lam, ctx.n)
        return gf, (gg if band.n_c else None), None, None, None, None, None, None


# ------------------------------------------------------------------ batches
class Batch:
    """Several bands solved together, one launch per kernel (cpm_batch_*):
    band i is solved with A_i = m[i] I + n[i] M_i, nrhs right-hand sides each.
    Batch vectors are (nrhs, total); instance i occupies columns
    offsets[i]:offsets[i+1]."""

    def __init__(self, bands, m, n, nrhs=1, allocator="torch"):
        self.handle = None
        bands, m, n = list(bands), list(m), list(n)
        if not bands or len(m) != len(bands) or len(n) != len(bands):
            raise ValueError("one (m, n) pair per band (got %d bands, %d m, %d n)"
                             % (len(bands), len(m), len(n)))
        if int(nrhs) < 1:
            raise ValueError("nrhs must be >= 1")
        lib = capi.load()
        self._lib = lib
        self.bands = bands                # keep the bands alive
        k = len(self.bands)
        arr = (C.c_void_p * k)(*[b.handle.value for b in self.bands])
        mm = (C.c_double * k)(*[float(x) for x in m])
        nn = (C.c_double * k)(*[float(x) for x in n])
        out = C.c_void_p()
        capi.check(lib.cpm_batch_create(arr, k, mm, nn, int(nrhs), _allocator(allocator),
                                        _stream(), C.byref(out)))
        self.handle = out
        _LIVE.add(self)
        self.nrhs = int(nrhs)
        offs = (C.c_int64 * (k + 1))()
        capi.check(lib.cpm_batch_offsets(self.handle, offs))
        self.offsets = list(offs)
        self.total = self.offsets[-1]

    def close(self):
        if self.handle is not None and self.handle.value:
            self._lib.cpm_batch_free(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, t):
        if not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != (self.nrhs, self.total):
            raise ValueError("batch vectors are contiguous GPU tensors of shape (%d, %d)"
                             % (self.nrhs, self.total))

    def apply(self, u):
        self._check(u)
        v = torch.empty_like(u)
        capi.check(self._lib.cpm_batch_apply(self.handle, _dtype_code(u), _ptr(u), _ptr(v),
                                             _stream()))
        return v

    def autotune(self, dtype=torch.float64, reps=5):
        ms = (C.c_double * capi.TUNE_VARIANTS)()
        best = C.c_int()
        code = capi.F64 if dtype == torch.float64 else capi.F32
        capi.check(self._lib.cpm_batch_autotune(self.handle, code, int(reps), _stream(), ms,
                                                C.byref(best)))
        return list(ms), best.value

    def solve(self, b, tol=1e-8, mode="mixed", x0=None, maxit=0, inner_tol=0.0,
              check_every=0, use_graph=True, raise_noconv=True):
        """Returns (x, stats) with one stats dict per system (r * nbands + i)."""
        self._check(b)
        if b.dtype != torch.float64:
            raise TypeError("right-hand sides are float64")
        if x0 is not None:
            _check_like(x0, b)
        x = torch.zeros_like(b) if x0 is None else x0.clone().contiguous()
        ns = self.nrhs * len(self.bands)
        st = (capi.SolveStats * ns)()
        o = _opts(0.0, 0.0, tol, mode, maxit, inner_tol, check_every, use_graph, 0.0)
        status = self._lib.cpm_batch_solve(self.handle, C.byref(o), _ptr(b), _ptr(x), st,
                                           _stream())
        stats = [{k: getattr(s, k) for k, _ in capi.SolveStats._fields_} for s in st]
        if not (status == capi.E_NOCONV and not raise_noconv):
            capi.check(status)
        return x, stats
