"""Failure handling of the solvers, forced from the host: non-finite data is
refused, a BiCGSTAB breakdown (rho = (r0_hat, r) = 0) restarts from the
current iterate with a new shadow residual (as the Eigen solver the paper
follows does, Sec. 5.4) and still converges to the same solution, and the
differentiable solve raises when either of its solves misses its
tolerance."""

import os

import numpy as np
import pytest

from paper_2305_04711_amd import capi

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


@pytest.fixture(scope="module")
def band(torch_cuda):
    from paper_2305_04711_amd import cpm
    return cpm.Band(cpm.sphere(), [cpm.latitude_ibc(0.3)], 24)


def _rhs(torch, band, seed=5):
    from paper_2305_04711_amd import cpm
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    f = torch.randn(band.n_s, dtype=torch.float64, device="cuda", generator=gen)
    g = torch.randn(band.n_c, dtype=torch.float64, device="cuda", generator=gen)
    return f, g, cpm.rhs(band, f, g, -1.0)


@pytest.mark.parametrize("mode", ["f64", "mixed", "gmres"])
def test_non_finite_data_is_refused(torch_cuda, band, mode):
    torch = torch_cuda
    from paper_2305_04711_amd import cpm
    f, g, b = _rhs(torch, band)
    f[17] = float("nan")
    bn = cpm.rhs(band, f, g, -1.0)
    with pytest.raises(capi.CPMError) as e:
        cpm.solve(band, bn, 0.0, -1.0, tol=1e-10, mode=mode)
    assert e.value.status == capi.E_INVALID and "right-hand side" in str(e.value)
    x0 = torch.zeros_like(b)
    x0[3] = float("inf")
    with pytest.raises(capi.CPMError) as e:
        cpm.solve(band, b, 0.0, -1.0, tol=1e-10, mode=mode, x0=x0)
    assert e.value.status == capi.E_INVALID and "initial guess" in str(e.value)
    with pytest.raises(capi.CPMError) as e:
        cpm.solve_adjoint(band, bn, 0.0, -1.0, tol=1e-10, mode="f64")
    assert e.value.status == capi.E_INVALID


def test_forced_breakdown_restarts_and_converges(torch_cuda, band):
    torch = torch_cuda
    from paper_2305_04711_amd import cpm
    f, g, b = _rhs(torch, band)
    x_ref, st_ref = cpm.solve(band, b, 0.0, -1.0, tol=1e-11, mode="f64")
    assert st_ref["restarts"] == 0
    os.environ["CPM_TEST_BREAKDOWN_AT"] = "40"
    try:
        x, st = cpm.solve(band, b, 0.0, -1.0, tol=1e-11, mode="f64", use_graph=False)
        xa, sta = cpm.solve_adjoint(band, b, 0.0, -1.0, tol=1e-11, mode="f64")
    finally:
        del os.environ["CPM_TEST_BREAKDOWN_AT"]
    print("forced breakdown:", st, sta, flush=True)
    assert st["restarts"] >= 1 and st["converged"] and st["relres"] <= 1e-11
    assert sta["restarts"] >= 1 and sta["converged"]
    err = (x - x_ref).abs().max().item() / x_ref.abs().max().item()
    assert err < 1e-6, err
    # the hook is read per solve: without it no restart happens
    x2, st2 = cpm.solve(band, b, 0.0, -1.0, tol=1e-11, mode="f64")
    assert st2["restarts"] == 0


def test_differentiable_solve_raises_when_a_solve_misses_tol(torch_cuda, band, monkeypatch):
    torch = torch_cuda
    from paper_2305_04711_amd import cpm
    f, g, _ = _rhs(torch, band)
    fr, gr = f.clone().requires_grad_(True), g.clone().requires_grad_(True)
    # below the FP64 residual floor: the forward solve cannot reach it
    with pytest.raises(capi.CPMError) as e:
        cpm.CPMSolve.apply(fr, gr, band, 0.0, -1.0, 1e-17, "f64")
    assert "forward solve" in str(e.value)
    stats = {}
    u = cpm.CPMSolve.apply(fr, gr, band, 0.0, -1.0, 1e-10, "f64", stats)
    assert stats["forward"]["relres"] <= 1e-10
    real = cpm.solve_adjoint

    def short(*a, **k):
        lam, st = real(*a, **k)
        st = dict(st, relres=10.0 * k["tol"], converged=0)
        return lam, st

    monkeypatch.setattr(cpm, "solve_adjoint", short)
    loss = (u ** 2).sum()
    with pytest.raises(capi.CPMError) as e:
        loss.backward()
    assert "adjoint solve" in str(e.value)
    assert stats["backward"]["relres"] > 1e-10
