"""cpm_apply_noalloc (the apply for callers that cannot allocate device
memory) against cpm_apply through the C ABI: the same kernels, so the same
result bit for bit, on two calls in a row (the second on a smaller band, so
the shared static scratch holds the first call's larger contents), in both
dtypes, and a clean refusal above the static scratch limit."""

import ctypes as C

import numpy as np
import pytest

from paper_2305_04711_amd import capi, cpm

pytestmark = pytest.mark.gpu

NOALLOC_MAX_ENTRIES = (32 << 20) // 8      # n * nrhs limit of the static scratch


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def _call(fn, band, u, m, n, torch):
    nrhs = 1 if u.dim() == 1 else u.shape[0]
    v = torch.full_like(u, float("nan"))
    code = capi.F64 if u.dtype == torch.float64 else capi.F32
    st = fn(band.handle, float(m), float(n), code, nrhs, C.c_void_p(u.data_ptr()),
            C.c_void_p(v.data_ptr()), C.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st, v


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_noalloc_apply_equals_apply_twice_shrinking(torch_cuda, dtype):
    torch = torch_cuda
    lib = capi.load()
    tdt = torch.float64 if dtype == "f64" else torch.float32
    big = cpm.Band(cpm.sphere(), [cpm.latitude_ibc(0.3)], 24)
    small = cpm.Band(cpm.circle(), [cpm.point_ibc((1.0, 0.0), (0.0, 1.0))], 32)
    assert small.n < big.n
    gen = torch.Generator(device="cuda")
    gen.manual_seed(11)
    cases = [(big, 2, 0.0, -1.0), (small, 1, 1.0, -0.5)]
    for band, nrhs, m, n in cases:
        print("noalloc case", dtype, "n", band.n, "nrhs", nrhs, flush=True)
        shape = (band.n,) if nrhs == 1 else (nrhs, band.n)
        u = torch.randn(shape, device="cuda", dtype=torch.float64, generator=gen).to(tdt)
        st_ref, v_ref = _call(lib.cpm_apply, band, u, m, n, torch)
        st_na, v_na = _call(lib.cpm_apply_noalloc, band, u, m, n, torch)
        torch.cuda.synchronize()
        assert st_ref == capi.OK, lib.cpm_last_error()
        assert st_na == capi.OK, lib.cpm_last_error()
        a, b = v_ref.cpu().numpy(), v_na.cpu().numpy()
        assert np.all(np.isfinite(b))
        rel = np.max(np.abs(a - b)) / np.max(np.abs(a))
        assert rel <= (1e-13 if dtype == "f64" else 2e-6), rel
        assert np.array_equal(a, b), "noalloc apply differs from cpm_apply (rel %.3g)" % rel


def test_noalloc_apply_refuses_above_the_static_limit(torch_cuda):
    torch = torch_cuda
    lib = capi.load()
    band = cpm.Band(cpm.sphere(), [], 64)
    nrhs = NOALLOC_MAX_ENTRIES // band.n + 1
    assert band.n * nrhs > NOALLOC_MAX_ENTRIES
    u = torch.zeros((nrhs, band.n), device="cuda", dtype=torch.float64)
    st, v = _call(lib.cpm_apply_noalloc, band, u, 0.0, -1.0, torch)
    torch.cuda.synchronize()
    assert st == capi.E_INVALID
    msg = lib.cpm_last_error().decode()
    assert "static limit" in msg and "4194304" in msg, msg
    assert torch.isnan(v).all(), "a refused call must enqueue nothing"
    # at the limit the same band is accepted
    nrhs_ok = NOALLOC_MAX_ENTRIES // band.n
    u2 = torch.randn((nrhs_ok, band.n), device="cuda", dtype=torch.float64)
    st2, v2 = _call(lib.cpm_apply_noalloc, band, u2, 0.0, -1.0, torch)
    st3, v3 = _call(lib.cpm_apply, band, u2, 0.0, -1.0, torch)
    torch.cuda.synchronize()
    assert st2 == capi.OK and st3 == capi.OK
    assert torch.equal(v2, v3)
