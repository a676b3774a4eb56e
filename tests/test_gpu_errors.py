"""Error behaviour of the C ABI (the status codes include/cpm.h documents),
and the degenerate inputs of the path: each call fails cleanly with its code
and a message, or returns the trivial answer, and the library stays usable."""

import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _status(fn):
    from paper_2305_04711_amd import capi
    try:
        fn()
    except capi.CPMError as e:
        return e.status, str(e)
    return capi.OK, ""


def test_build_band_rejects_bad_grids_and_boundaries():
    from paper_2305_04711_amd import capi, cpm
    cases = [
        lambda: cpm.Band(cpm.sphere(), [], 0),                       # N <= 0
        lambda: cpm.Band(cpm.sphere(), [], 16, p=4),                 # degree
        lambda: cpm.Band(cpm.sphere(), [], 16, order=3),             # IBC order
        lambda: cpm.Band(cpm.sphere(), [cpm.meridian_ibc(1.0, 0.0)], 16),   # kind/surface
        lambda: cpm.Band(cpm.torus(1.0, 0.4), [cpm.latitude_ibc(0.3)], 16),   # kind/surface
    ]
    for k, fn in enumerate(cases):
        st, msg = _status(fn)
        assert st == capi.E_INVALID, (k, st, msg)
        assert msg
    # a zero-Neumann condition at a point of a surface is not defined
    ib = cpm.point_ibc((0.0, 0.0, 1.0), (1.0, 0.0, 0.0))
    ib.bc[0] = capi.BC_NEUMANN
    st, msg = _status(lambda: cpm.Band(cpm.sphere(), [ib], 16))
    assert st == capi.E_INVALID and "Neumann" in msg


def test_narrow_band_reports_stencil_holes():
    """A band of radius 2.5h cannot hold a cubic stencil (reading 1)."""
    from paper_2305_04711_amd import capi, cpm
    st, msg = _status(lambda: cpm.Band(cpm.sphere(), [], 32, r_band=2.5 / 32))
    assert st == capi.E_STENCIL_HOLE, (st, msg)
    assert "not band nodes" in msg


def test_reach_bound():
    """h too coarse for the torus tube (r = sqrt(17) h above rho)."""
    from paper_2305_04711_amd import capi, cpm
    st, msg = _status(lambda: cpm.Band(cpm.torus(1.0, 0.4), [], 8, check_reach=True))
    assert st == capi.E_REACH, (st, msg)
    band = cpm.Band(cpm.torus(1.0, 0.4), [], 32, check_reach=True)
    assert band.n > 0


def test_overlapping_check_regions():
    from paper_2305_04711_amd import capi, cpm
    st, msg = _status(lambda: cpm.Band(cpm.sphere(), [cpm.latitude_ibc(0.3),
                                                      cpm.latitude_ibc(0.32)], 32))
    assert st == capi.E_OVERLAP, (st, msg)


def test_vector_arguments_are_checked():
    import torch
    from paper_2305_04711_amd import capi, cpm
    band = cpm.Band(cpm.sphere(), [cpm.latitude_ibc(0.3)], 16)
    lib, h = band._lib, band.handle
    u = torch.zeros(band.n, device="cuda", dtype=torch.float64)
    v = torch.empty_like(u)
    vp = lambda t: C.c_void_p(t.data_ptr())
    assert lib.cpm_apply(h, 0.0, -1.0, 0, 1, None, vp(v), None) == capi.E_INVALID
    assert lib.cpm_apply(h, 0.0, -1.0, 7, 1, vp(u), vp(v), None) == capi.E_INVALID
    assert lib.cpm_apply(h, 0.0, -1.0, 0, 0, vp(u), vp(v), None) == capi.E_INVALID
    assert lib.cpm_apply(h, 0.0, -1.0, 0, 1, vp(u), vp(u), None) == capi.E_INVALID
    assert lib.cpm_apply_transpose(None, 0.0, -1.0, 0, 1, vp(u), vp(v), None) == capi.E_INVALID
    assert lib.cpm_last_error()
    with pytest.raises((ValueError, TypeError)):
        cpm.apply(band, torch.zeros(band.n + 1, device="cuda", dtype=torch.float64), 0.0, -1.0)
    with pytest.raises((ValueError, TypeError)):
        cpm.apply(band, torch.zeros(band.n, dtype=torch.float64), 0.0, -1.0)   # host tensor
    # the band still works after the rejected calls
    assert lib.cpm_apply(h, 0.0, -1.0, 0, 1, vp(u), vp(v), None) == capi.OK
    torch.cuda.synchronize()
    assert float(v.abs().max()) == 0.0


def test_binding_checks_arguments_before_the_library_reads_them():
    """Shapes and dtypes the kernels would read past (a float32 vector read as
    double, fewer rows of g than of f, a warm start of another shape) are
    refused by the binding before any call into the library."""
    import torch
    from paper_2305_04711_amd import cpm
    band = cpm.Band(cpm.sphere(), [cpm.latitude_ibc(0.3)], 16)
    dev = "cuda"
    f = torch.zeros(2, band.n_s, dtype=torch.float64, device=dev)
    g = torch.zeros(2, band.n_c, dtype=torch.float64, device=dev)
    with pytest.raises(TypeError):
        cpm.rhs(band, f.float(), g, -1.0)
    with pytest.raises(TypeError):
        cpm.rhs(band, f, g.float(), -1.0)
    with pytest.raises(ValueError):
        cpm.rhs(band, f, g[0].contiguous(), -1.0)
    with pytest.raises(ValueError):
        cpm.rhs(band, f, None, -1.0)
    with pytest.raises(TypeError):
        cpm.rhs_adjoint(band, torch.zeros(band.n, dtype=torch.float32, device=dev), -1.0)
    with pytest.raises(ValueError):
        cpm.apply(band, torch.zeros(1, 2, band.n, dtype=torch.float64, device=dev), 0.0, -1.0)
    b = torch.ones(band.n, dtype=torch.float64, device=dev)
    for x0 in (torch.zeros(band.n + 1, dtype=torch.float64, device=dev),
               torch.zeros(band.n, dtype=torch.float32, device=dev),
               torch.zeros(1, band.n, dtype=torch.float64, device=dev)):
        with pytest.raises(ValueError):
            cpm.solve(band, b, 0.0, -1.0, x0=x0)
    # the same calls with matching arguments go through
    assert cpm.rhs(band, f, g, -1.0).shape == (2, band.n)
    x, st = cpm.solve(band, b, 1.0, -1.0, tol=1e-8, mode="f64", x0=torch.zeros_like(b))
    assert st["converged"]


@pytest.mark.parametrize("mode", ["f64", "mixed"])
def test_solve_edge_cases(mode):
    """A zero right-hand side returns x = 0 at once; a maxit too small for the
    tolerance raises CPM_E_NOCONV, or returns its best iterate (residual not
    above the starting one) when asked not to raise."""
    import torch
    from paper_2305_04711_amd import capi, cpm
    band = cpm.Band(cpm.sphere(), [cpm.latitude_ibc(0.3)], 24)
    z = torch.zeros(band.n, device="cuda", dtype=torch.float64)
    x, st = cpm.solve(band, z, 0.0, -1.0, tol=1e-10, mode=mode)
    assert st["converged"] and float(x.abs().max()) == 0.0
    rng = np.random.default_rng(4)
    b = torch.tensor(rng.standard_normal(band.n), device="cuda")
    st_code, msg = _status(lambda: cpm.solve(band, b, 0.0, -1.0, tol=1e-12, mode=mode, maxit=5))
    assert st_code == capi.E_NOCONV, (st_code, msg)
    x, st = cpm.solve(band, b, 0.0, -1.0, tol=1e-12, mode=mode, maxit=5, raise_noconv=False)
    assert not st["converged"]
    assert st["relres"] <= 1.0 and torch.isfinite(x).all()
