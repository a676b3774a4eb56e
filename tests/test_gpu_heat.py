"""Crank-Nicolson time stepping on the GPU (cpm_heat_cn): the heat test of
Sec. 6.2 on the unit sphere, exact solution exp(-2t) x_axis, with a Dirichlet
latitude IBC (data = the exact solution on C) or a zero-Neumann equator IBC.

  * parity with the oracle's Crank-Nicolson (oracle.timestep) on small bands;
  * second-order convergence of the paper's run (dt = 0.1 h to t = 0.1) to
    the closed form, on grid values of nodes whose FD neighbours are all in
    the band, away from C.
"""

import numpy as np
import pytest

from closed_forms import heat_l1
from oracle import geometry as G
from oracle import timestep as TS
from parity_helpers import dof_map, oracle_and_gpu

pytestmark = pytest.mark.gpu


def _setup(cp, bc_cpc, bc_node, n_s, n_c, N, T, axis):
    dt = 0.1 / N
    nsteps = int(round(T / dt))
    u0 = np.empty(n_s + n_c)
    u0[:n_s] = heat_l1(cp, 0.0, axis)
    u0[n_s:] = u0[bc_node]
    g = np.stack([heat_l1(bc_cpc, k * dt, axis) for k in range(nsteps + 1)]) if n_c else None
    return dt, nsteps, u0, g


@pytest.mark.parametrize("cfg,axis", [("sphere_lat", 2), ("sphere_eq_neumann", 0)])
def test_heat_cn_matches_oracle(cfg, axis):
    import torch
    from paper_2305_04711_amd import cpm
    N = 16
    sysm, band = oracle_and_gpu(cfg, N)
    g2o = dof_map(sysm, band)
    dt, nsteps, u0, g = _setup(sysm.CP, sysm.bc_cpc, sysm.bc_node, sysm.n_s, sysm.n_c, N, 0.025, axis)
    ref = TS.heat_cn(sysm, u0, dt, nsteps, g)
    gg = torch.tensor(g[:, g2o[band.n_s:] - sysm.n_s].copy(), device="cuda")
    u, st = cpm.heat_cn(band, torch.tensor(u0[g2o], device="cuda"), dt, nsteps, gg, tol=1e-13)
    err = np.max(np.abs(u.cpu().numpy() - ref[g2o])) / np.max(np.abs(ref))
    print(cfg, "steps", nsteps, st, "rel err", err, flush=True)
    assert st["converged"] and err < 1e-9


@pytest.mark.parametrize("bc,z0,axis", [("dirichlet", 0.3, 2), ("neumann", 0.0, 0)])
def test_heat_paper_run_second_order(bc, z0, axis):
    import torch
    from paper_2305_04711_amd import cpm
    errs = []
    for N in (32, 64):
        band = cpm.Band(cpm.sphere(), [cpm.latitude_ibc(z0, bc=bc)], N, order=2)
        cp = band.cp()
        dt, nsteps, u0, g = _setup(cp, band.bc_cpc(), band.bc_node(), band.n_s, band.n_c, N,
                                   0.1, axis)
        u, st = cpm.heat_cn(band, torch.tensor(u0, device="cuda"), dt, nsteps,
                            torch.tensor(g, device="cuda"), tol=1e-12)
        assert st["converged"]
        X = band.coords() / float(N)
        depth = np.abs(np.sqrt((X * X).sum(1)) - 1.0)
        keep = (depth <= np.sqrt(17.0) / N - 1.0 / N) & (np.abs(cp[:, 2] - z0) > 0.2)
        T = nsteps * dt
        errs.append(np.max(np.abs(u.cpu().numpy()[:band.n_s][keep] - heat_l1(cp[keep], T, axis))))
        print(bc, N, "steps", nsteps, "Linf", errs[-1], st, flush=True)
    assert np.log2(errs[0] / errs[1]) > 1.7, errs
