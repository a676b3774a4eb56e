"""The stencil-set band (Sec. 5.1 cites it: only the nodes interpolation and
FD stencils need) on the GPU against the oracle's: node sets, closest points,
stencil indices bit for bit, the operator, its transpose, the right-hand side
and the solves, in 2-D and 3-D with interior boundaries; and its size against
the tube's."""

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spl

from oracle import adjoint as AD
from parity_helpers import NEUMANN_CASES, dof_map, oracle_and_gpu

pytestmark = pytest.mark.gpu

CASES = [("circle_point", 40), ("sphere_lat", 20), ("torus_meridians", 16),
         ("sphere_eq_neumann", 18), ("sphere_arc", 24)]
_cache = {}


def _pair(cfg, N, degree=3):
    if (cfg, N, degree) not in _cache:
        sysm, band = oracle_and_gpu(cfg, N, order=2, degree=degree, band="stencil_set")
        _cache[(cfg, N, degree)] = (sysm, band, dof_map(sysm, band))
    return _cache[(cfg, N, degree)]


def _pattern(r, c, n):
    return sp.csr_matrix((np.ones(len(r)), (r, c)), shape=(n, n)).astype(bool).astype(np.int8)


@pytest.mark.parametrize("cfg,N", CASES + [("sphere_lat", 16)])
def test_stencil_set_sets_and_stencils_bit_exact(cfg, N):
    degree = 2 if N == 16 and cfg == "sphere_lat" else 3
    sysm, band, g2o = _pair(cfg, N, degree)
    assert band.n_s == sysm.n_s and band.n_c == sysm.n_c
    cp = band.cp()
    assert np.array_equal(cp.view(np.uint64), sysm.CP[g2o[:band.n_s]].view(np.uint64))
    n = band.n
    ec = band.ecols()
    r, o = np.nonzero(ec >= 0)
    E = sysm.E.tocoo()
    D = _pattern(g2o[r], g2o[ec[r, o]], n) - _pattern(E.row, E.col, n)
    D.eliminate_zeros()
    assert D.nnz == 0
    lc = band.lcols()
    r, o = np.nonzero(lc >= 0)
    L = sysm.L_off.tocoo()
    D = _pattern(g2o[r], g2o[lc[r, o]], n) - _pattern(L.row, L.col, n)
    D.eliminate_zeros()
    assert D.nnz == 0


@pytest.mark.parametrize("cfg,N", CASES)
def test_stencil_set_apply_transpose_rhs_match_oracle(cfg, N):
    import torch
    from paper_2305_04711_amd import cpm
    sysm, band, g2o = _pair(cfg, N)
    rng = np.random.default_rng(18)
    U = rng.standard_normal((2, sysm.n))
    m, n = 0.5, -1.0
    for td, tol in ((torch.float64, 1e-13), (torch.float32, 2e-6)):
        u = torch.tensor(U[:, g2o], dtype=td, device="cuda").contiguous()
        for fn, ref in ((cpm.apply, np.stack([sysm.apply(U[r], m, n) for r in range(2)])),
                        (cpm.apply_transpose,
                         np.stack([AD.apply_transpose(sysm, U[r], m, n) for r in range(2)]))):
            v = fn(band, u, m, n).cpu().numpy().astype(np.float64)
            err = np.max(np.abs(v - ref[:, g2o])) / np.max(np.abs(ref))
            assert err < tol, (fn.__name__, td, err)
    if sysm.n_c:
        f_o = rng.standard_normal(sysm.n_s)
        g_o = rng.standard_normal(sysm.n_c)
        ref = sysm.rhs(f_o, g_o, n)
        b = cpm.rhs(band, torch.tensor(f_o[g2o[:band.n_s]], device="cuda"),
                    torch.tensor(g_o[g2o[band.n_s:] - sysm.n_s], device="cuda"), n).cpu().numpy()
        assert np.max(np.abs(b - ref[g2o])) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("mode", ["f64", "mixed"])
@pytest.mark.parametrize("cfg,N", [("circle_point", 32), ("sphere_lat", 16), ("sphere_eq_neumann", 16)])
def test_stencil_set_solve_matches_oracle(cfg, N, mode):
    import torch
    from paper_2305_04711_amd import cpm
    sysm, band, g2o = _pair(cfg, N)
    rng = np.random.default_rng(19)
    f_o = rng.standard_normal(sysm.n_s)
    g_o = rng.standard_normal(sysm.n_c)
    m, n = (1.0, -1.0) if cfg in NEUMANN_CASES else (0.0, -1.0)
    b_o = sysm.rhs(f_o, g_o, n)
    x_o = spl.spsolve(sysm.matrix(m, n).tocsc(), b_o)
    x, st = cpm.solve(band, torch.tensor(b_o[g2o], device="cuda"), m, n, tol=1e-12, mode=mode)
    assert st["converged"]
    err = np.max(np.abs(x.cpu().numpy() - x_o[g2o])) / np.max(np.abs(x_o))
    print("stencil-set solve", cfg, N, mode, st, "relLinf", err, flush=True)
    assert err < 1e-6


def test_stencil_set_is_smaller_than_the_tube_at_full_size():
    """The torus with two meridian IBCs at h = 1/512: the stencil set keeps a
    subset of the tube's nodes (every kept node is a tube node with the same
    stored cp_S), 6-15% smaller."""
    import torch
    from paper_2305_04711_amd import cpm
    ib = [cpm.meridian_ibc(1.0, 0.0), cpm.meridian_ibc(-1.0, 0.0)]
    tube = cpm.Band(cpm.torus(1.0, 0.4), ib, 512)
    ss = cpm.Band(cpm.torus(1.0, 0.4), ib, 512, band="stencil_set")
    red = 1.0 - ss.n / tube.n
    print("torus h=1/512: tube", tube.n, "stencil set", ss.n, "reduction", red, flush=True)
    assert 0.06 <= red <= 0.15
    K1, K2 = tube.coords().astype(np.int64), ss.coords().astype(np.int64)
    off = 1 << 20
    key = lambda K: ((K[:, 0] + off) << 42) | ((K[:, 1] + off) << 21) | (K[:, 2] + off)
    k1, k2 = key(K1), key(K2)
    order = np.argsort(k1)
    pos = np.searchsorted(k1[order], k2)
    assert np.all(k1[order][np.minimum(pos, k1.size - 1)] == k2)
    cp1, cp2 = tube.cp(), ss.cp()
    assert np.array_equal(cp1[order][pos].view(np.uint64), cp2.view(np.uint64))
    u = torch.randn(ss.n, device="cuda", dtype=torch.float64)
    v = cpm.apply(ss, u, 0.0, -1.0)
    assert torch.isfinite(v).all()
