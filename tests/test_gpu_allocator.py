"""The caller's allocator at the C ABI: every device allocation of a band or
batch goes through the cpm_allocator given at creation (the torch caching
allocator from the Python binding), is counted by torch, and is returned at
free; a failing allocator yields CPM_E_OOM with every block it gave back."""

import ctypes as C

import numpy as np
import pytest

from paper_2305_04711_amd import capi, cpm

pytestmark = pytest.mark.gpu


def _slack(nbytes):
    """Bytes the torch caching allocator may count above the requested ones:
    blocks are rounded to 512 bytes, and a large block is not split when the
    rest would be under 1 MiB, so the whole block counts."""
    return 0.10 * nbytes + (4 << 20)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def test_band_memory_comes_from_torch_and_returns(torch_cuda):
    torch = torch_cuda
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    band = cpm.Band(cpm.sphere(), [cpm.latitude_ibc(0.3)], 32)
    torch.cuda.synchronize()
    arrays, scratch = band.memory()
    grown = torch.cuda.memory_allocated() - base
    print("band arrays", arrays, "torch growth", grown, flush=True)
    assert scratch == 0
    assert arrays <= grown <= arrays + _slack(arrays)
    # an apply and a solve grow the band's scratch through the same pool
    u = torch.randn(band.n, dtype=torch.float64, device="cuda")
    v = cpm.apply(band, u, 0.0, -1.0)
    x, st = cpm.solve(band, v, 0.0, -1.0, tol=1e-10, mode="mixed")
    torch.cuda.synchronize()
    arrays2, scratch2 = band.memory()
    assert arrays2 == arrays and scratch2 >= 8 * band.n
    held = torch.cuda.memory_allocated() - base - (u.numel() + v.numel() + x.numel()) * 8
    assert arrays + scratch2 <= held <= arrays + scratch2 + _slack(arrays + scratch2)
    del x, v, u
    band.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == base


def test_hipmalloc_band_is_invisible_to_torch_and_computes_the_same(torch_cuda):
    torch = torch_cuda
    gen = torch.Generator(device="cuda")
    gen.manual_seed(3)
    bt = cpm.Band(cpm.torus(1.0, 0.4), [cpm.meridian_ibc(1.0, 0.0)], 24)
    u = torch.randn(bt.n, dtype=torch.float64, device="cuda", generator=gen)
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    bh = cpm.Band(cpm.torus(1.0, 0.4), [cpm.meridian_ibc(1.0, 0.0)], 24, allocator=None)
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == base
    assert bh.memory()[0] == bt.memory()[0]
    for dt in (torch.float64, torch.float32):
        a = cpm.apply(bt, u.to(dt), 0.0, -1.0)
        b = cpm.apply(bh, u.to(dt), 0.0, -1.0)
        assert torch.equal(a, b)
        a = cpm.apply_transpose(bt, u.to(dt), 1.0, -0.5)
        b = cpm.apply_transpose(bh, u.to(dt), 1.0, -0.5)
        assert torch.equal(a, b)
    bh.close()
    bt.close()


def test_batch_memory_comes_from_torch_and_returns(torch_cuda):
    torch = torch_cuda
    bands = [cpm.Band(cpm.sphere(), [], 20), cpm.Band(cpm.torus(1.0, 0.4), [], 24)]
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    batch = cpm.Batch(bands, [1.0, 1.0], [-1.0, -1.0], nrhs=2)
    batch.autotune(torch.float64, reps=1)
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() > base
    batch.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == base


class _Counting:
    """An allocator over the torch pool that fails after `limit` blocks."""

    def __init__(self, torch, limit):
        self.torch, self.limit, self.live, self.calls = torch, limit, {}, 0
        self.alloc_fn = capi.ALLOC_FN(self._alloc)
        self.free_fn = capi.FREE_FN(self._free)
        self.st = capi.Allocator(self.alloc_fn, self.free_fn, None)

    def _alloc(self, nbytes, stream, ctx):
        self.calls += 1
        if self.calls > self.limit:
            return 0
        p = int(self.torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0)))
        self.live[p] = int(nbytes)
        return p

    def _free(self, ptr, nbytes, stream, ctx):
        assert self.live.pop(int(ptr)) == int(nbytes)
        self.torch.cuda.caching_allocator_delete(int(ptr))


def test_failing_allocator_gives_oom_and_returns_every_block(torch_cuda):
    torch = torch_cuda
    lib = capi.load()
    grid = capi.Grid(24, 3, 2, 0, 0.0, 0.0, 0.0, capi.BAND_TUBE)
    surf = cpm.sphere()
    ib = (capi.IBC * 1)(cpm.latitude_ibc(0.3))
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    # count the allocations of a full build, then fail at several points of it
    full = _Counting(torch, 10 ** 9)
    out = C.c_void_p()
    assert lib.cpm_build_band(C.byref(surf), ib, 1, C.byref(grid), C.byref(full.st), stream,
                              C.byref(out)) == capi.OK
    n_full = full.calls
    lib.cpm_band_free(out)
    assert not full.live and n_full > 10
    for limit in (0, 3, n_full // 2, n_full - 1):
        al = _Counting(torch, limit)
        out = C.c_void_p()
        st = lib.cpm_build_band(C.byref(surf), ib, 1, C.byref(grid), C.byref(al.st), stream,
                                C.byref(out))
        print("allocator limit", limit, "status", st, flush=True)
        assert st == capi.E_OOM and not out.value
        assert b"allocator returned NULL" in lib.cpm_last_error()
        assert not al.live, "blocks not returned after a failed build: %d" % len(al.live)
    # an allocator without free is refused before anything is allocated
    half = capi.Allocator(full.alloc_fn, capi.FREE_FN(), None)
    assert lib.cpm_build_band(C.byref(surf), ib, 1, C.byref(grid), C.byref(half), stream,
                              C.byref(out)) == capi.E_INVALID
