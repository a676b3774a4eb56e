"""Quadratic interpolation (p = 2, Sec. 7) on the GPU against the oracle:
band sets (radius from eq. (bandwidth) with p = 2), nearest-node stencil
bases and member indices bit for bit, the operator, its transpose, the
right-hand side and the solves, in 2-D and 3-D with interior boundaries."""

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spl

from oracle import adjoint as AD
from parity_helpers import NEUMANN_CASES, dof_map, oracle_and_gpu

pytestmark = pytest.mark.gpu

CASES = [("circle_point", 40), ("sphere_lat", 20), ("torus_meridians", 18),
         ("sphere_eq_neumann", 18)]
_cache = {}


def _pair(cfg, N):
    if (cfg, N) not in _cache:
        sysm, band = oracle_and_gpu(cfg, N, order=2, degree=2)
        _cache[(cfg, N)] = (sysm, band, dof_map(sysm, band))
    return _cache[(cfg, N)]


def _pattern(r, c, n):
    return sp.csr_matrix((np.ones(len(r)), (r, c)), shape=(n, n)).astype(bool).astype(np.int8)


@pytest.mark.parametrize("cfg,N", CASES)
def test_quadratic_band_and_stencils_bit_exact(cfg, N):
    sysm, band, g2o = _pair(cfg, N)
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
    base = band.bases()[:band.n_s]
    S = sysm.CP[g2o[:band.n_s]] * float(N)
    assert np.array_equal(base, np.floor(S + 0.5).astype(np.int64) - 1)


@pytest.mark.parametrize("cfg,N", CASES)
def test_quadratic_apply_transpose_rhs_match_oracle(cfg, N):
    import torch
    from paper_2305_04711_amd import cpm
    sysm, band, g2o = _pair(cfg, N)
    rng = np.random.default_rng(16)
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
    f_o = rng.standard_normal(sysm.n_s)
    g_o = rng.standard_normal(sysm.n_c)
    ref = sysm.rhs(f_o, g_o, n)
    b = cpm.rhs(band, torch.tensor(f_o[g2o[:band.n_s]], device="cuda"),
                torch.tensor(g_o[g2o[band.n_s:] - sysm.n_s], device="cuda"), n).cpu().numpy()
    assert np.max(np.abs(b - ref[g2o])) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("mode", ["f64", "mixed"])
@pytest.mark.parametrize("cfg,N", [("circle_point", 32), ("sphere_lat", 16), ("sphere_eq_neumann", 16)])
def test_quadratic_solve_matches_oracle(cfg, N, mode):
    import torch
    from paper_2305_04711_amd import cpm
    sysm, band, g2o = _pair(cfg, N) if (cfg, N) in CASES else (None, None, None)
    if sysm is None:
        sysm, band = oracle_and_gpu(cfg, N, order=2, degree=2)
        g2o = dof_map(sysm, band)
    rng = np.random.default_rng(17)
    f_o = rng.standard_normal(sysm.n_s)
    g_o = rng.standard_normal(sysm.n_c)
    m, n = (1.0, -1.0) if cfg in NEUMANN_CASES else (0.0, -1.0)
    b_o = sysm.rhs(f_o, g_o, n)
    x_o = spl.spsolve(sysm.matrix(m, n).tocsc(), b_o)
    x, st = cpm.solve(band, torch.tensor(b_o[g2o], device="cuda"), m, n, tol=1e-12, mode=mode)
    assert st["converged"]
    err = np.max(np.abs(x.cpu().numpy() - x_o[g2o])) / np.max(np.abs(x_o))
    print("quadratic solve", cfg, N, mode, st, "relLinf", err, flush=True)
    assert err < 1e-6
