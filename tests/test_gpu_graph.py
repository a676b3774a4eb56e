"""Graph replay against eager launches.  The solvers capture blocks of
iterations into HIP graphs and replay them many times, with host reads and
eager kernels (residual replacements, restarts) between the replays.  Every
reduction and every scatter (the transposed explicit rows go through pull
lists) has a fixed summation order, so a solve with graphs must reproduce
the eager solve bit for bit, adjoint solves included."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _band(kind):
    from paper_2305_04711_amd import cpm
    if kind == "sphere_lat":
        return cpm.Band(cpm.sphere(), [cpm.latitude_ibc(0.3)], 24)
    return cpm.Band(cpm.torus(1.0, 0.4), [cpm.meridian_ibc(1.0, 0.0),
                                          cpm.meridian_ibc(-1.0, 0.0)], 24)


@pytest.mark.parametrize("kind", ["sphere_lat", "torus_meridians"])
@pytest.mark.parametrize("mode", ["f64", "mixed"])
def test_solve_graph_replays_equal_eager(kind, mode):
    import torch
    from paper_2305_04711_amd import cpm
    band = _band(kind)
    rng = np.random.default_rng(31)
    b = torch.tensor(rng.standard_normal(band.n), device="cuda")
    xg, sg = cpm.solve(band, b, 0.0, -1.0, tol=1e-10, mode=mode, use_graph=True)
    xe, se = cpm.solve(band, b, 0.0, -1.0, tol=1e-10, mode=mode, use_graph=False)
    # the graph is replayed many times (16 iterations per replay)
    assert sg["krylov_iters"] >= 64
    assert sg["krylov_iters"] == se["krylov_iters"]
    assert torch.equal(xg, xe)
    # and a second graph solve on the same band (cached executable) again
    xg2, _ = cpm.solve(band, b, 0.0, -1.0, tol=1e-10, mode=mode, use_graph=True)
    assert torch.equal(xg2, xe)


def test_gauged_solve_graph_equals_eager():
    import torch
    from paper_2305_04711_amd import cpm
    band = cpm.Band(cpm.sphere(), [], 20)
    rng = np.random.default_rng(32)
    b = torch.tensor(rng.standard_normal(band.n), device="cuda")
    b -= b.mean()
    g = float(band.N) ** 2
    xg, _ = cpm.solve(band, b, 0.0, -1.0, tol=1e-10, mode="f64", gauge=g, use_graph=True)
    xe, _ = cpm.solve(band, b, 0.0, -1.0, tol=1e-10, mode="f64", gauge=g, use_graph=False)
    assert torch.equal(xg, xe)


@pytest.mark.parametrize("mode", ["f64", "mixed"])
def test_adjoint_solve_graph_equals_eager(mode):
    import torch
    from paper_2305_04711_amd import cpm
    band = _band("torus_meridians")
    rng = np.random.default_rng(33)
    w = torch.tensor(rng.standard_normal(band.n), device="cuda")
    lg, sg = cpm.solve_adjoint(band, w, 0.0, -1.0, tol=1e-10, mode=mode, use_graph=True)
    le, se = cpm.solve_adjoint(band, w, 0.0, -1.0, tol=1e-10, mode=mode, use_graph=False)
    assert sg["converged"] and se["converged"]
    assert sg["krylov_iters"] == se["krylov_iters"]
    assert torch.equal(lg, le)


@pytest.mark.parametrize("mode", ["f64", "mixed"])
def test_batched_solve_graph_equals_eager(mode):
    import torch
    from paper_2305_04711_amd import cpm
    bands = [cpm.Band(cpm.sphere(), [], 16), cpm.Band(cpm.torus(1.0, 0.4), [], 20),
             cpm.Band(cpm.sphere(), [], 24)]
    batch = cpm.Batch(bands, [1.0] * 3, [-1.0] * 3, nrhs=2)
    rng = np.random.default_rng(34)
    b = torch.tensor(rng.standard_normal((2, batch.total)), device="cuda")
    xg, sg = batch.solve(b, tol=1e-10, mode=mode, use_graph=True)
    xe, se = batch.solve(b, tol=1e-10, mode=mode, use_graph=False)
    assert all(s["converged"] for s in sg)
    assert [s["krylov_iters"] for s in sg] == [s["krylov_iters"] for s in se]
    assert torch.equal(xg, xe)
