"""The HIP path at the full sizes of the target configurations: the sphere
with a latitude interior boundary at h = 1/256 (6.9M DOFs) and the torus with
two meridian boundaries at h = 1/512 (34.2M DOFs), in the launch
configuration bench.py times (autotuned apply).

At these sizes the oracle cannot assemble E and L, so:
  * band membership is checked at every node (bit-exact cp_S and distance),
    and closed under face neighbours (no missing node next to the band);
  * the apply is checked row by row on sampled rows (random rows, rows near
    the interior boundary where stencils are swapped, BC rows) against
    ``oracle.local``, which evaluates the paper's definitions per row;
  * the solve is checked by the residual of sampled rows computed by the
    oracle, and against the closed-form solution.
"""

import numpy as np
import pytest

from closed_forms import latitude_harmonic
from oracle import geometry as G
from oracle import local as LO
from paper_2305_04711_amd import capi, inputs

pytestmark = pytest.mark.gpu

OFF = 1 << 20


def _keys(K):
    K = np.asarray(K, dtype=np.int64) + OFF
    return (K[:, 0] << 42) | (K[:, 1] << 21) | (K[:, 2] if K.shape[1] == 3 else 0)


class GpuIndex:
    """(coords, curve) -> GPU DOF, for feeding GPU vectors to the oracle."""

    def __init__(self, band):
        self.K = band.coords().astype(np.int64)
        k = _keys(self.K)
        self.order = np.argsort(k)
        self.sk = k[self.order]
        self.n_s = band.n_s
        self.bc = {}
        if band.n_c:
            node, curve = band.bc_node(), band.bc_curve()
            for c in np.unique(curve):
                sel = np.nonzero(curve == c)[0]
                idx = np.full(band.n_s, -1, dtype=np.int64)
                idx[node[sel]] = band.n_s + sel
                self.bc[int(c)] = idx

    def pde(self, K):
        k = _keys(K)
        p = np.searchsorted(self.sk, k)
        p = np.minimum(p, self.sk.size - 1)
        ok = self.sk[p] == k
        out = np.where(ok, self.order[p], -1)
        return out

    def dof(self, K, curve):
        d = self.pde(K)
        assert np.all(d >= 0), "a node the oracle needs is missing from the GPU band"
        out = d.copy()
        for c, idx in self.bc.items():
            m = curve == c
            if m.any():
                a = idx[d[m]]
                assert np.all(a >= 0), "missing BC DOF"
                out[m] = a
        return out


_cache = {}


def _setup(name):
    if name in _cache:
        return _cache[name]
    import torch
    from paper_2305_04711_amd import cpm
    assert torch.cuda.is_available()
    if name == "torus_meridians_1024":
        S = G.Torus(1.0, 0.4)
        Cs = [G.MeridianC(S, 1.0, 0.0), G.MeridianC(S, -1.0, 0.0)]
        band = cpm.Band(cpm.torus(1.0, 0.4), [cpm.meridian_ibc(1.0, 0.0),
                                              cpm.meridian_ibc(-1.0, 0.0)], 1024)
        N = 1024
    elif name == "sphere_lat_256":
        S = G.Sphere()
        Cs = [G.LatitudeC(S, 0.3)]
        band = cpm.Band(cpm.sphere(), [cpm.latitude_ibc(0.3)], 256)
        N = 256
    else:
        S = G.Torus(1.0, 0.4)
        Cs = [G.MeridianC(S, 1.0, 0.0), G.MeridianC(S, -1.0, 0.0)]
        band = cpm.Band(cpm.torus(1.0, 0.4), [cpm.meridian_ibc(1.0, 0.0),
                                              cpm.meridian_ibc(-1.0, 0.0)], 512)
        N = 512
    cpm.autotune(band, torch.float64)
    cpm.autotune(band, torch.float32)
    ix = GpuIndex(band)
    loc = LO.LocalCPM(S, N, Cs)
    _cache[name] = (S, Cs, N, band, ix, loc)
    print("setup", name, "n_s", band.n_s, "n_c", band.n_c, flush=True)
    return _cache[name]


def _samples(S, Cs, N, band, ix, rng):
    K = ix.K
    r = np.sqrt(17.0) / N
    pick = rng.choice(band.n_s, 3000, replace=False)
    X = K / float(N)
    near = np.zeros(band.n_s, bool)
    for C in Cs:
        sub = np.unique(rng.integers(0, band.n_s, 4_000_000))
        dC = np.linalg.norm(X[sub] - C.cp(X[sub]), axis=1)
        near[sub[dC < 2 * r]] = True
    near_idx = np.nonzero(near)[0]
    pick_near = rng.choice(near_idx, min(3000, near_idx.size), replace=False)
    rows = np.concatenate([pick, pick_near])
    Ks = K[rows]
    curve = np.full(rows.size, -1)
    gpu_rows = rows.copy()
    if band.n_c:
        bsel = rng.choice(band.n_c, min(1500, band.n_c), replace=False)
        node = band.bc_node()[bsel]
        Ks = np.concatenate([Ks, K[node]])
        curve = np.concatenate([curve, band.bc_curve()[bsel]])
        gpu_rows = np.concatenate([gpu_rows, band.n_s + bsel])
    return Ks, curve, gpu_rows


@pytest.mark.parametrize("name", ["sphere_lat_256", "torus_meridians_512"])
def test_fullsize_band_membership(name):
    S, Cs, N, band, ix, loc = _setup(name)
    K = ix.K
    X = K / float(N)
    cp = band.cp()
    r = np.sqrt(17.0) / N
    # stored cp_S: the same formula, bit for bit
    assert np.array_equal(cp.view(np.uint64), S.cp(X).view(np.uint64))
    D = X - cp
    dist = np.sqrt((D[:, 0] * D[:, 0] + D[:, 1] * D[:, 1]) + D[:, 2] * D[:, 2])
    assert np.all(dist <= r)
    # closed under face neighbours: every absent neighbour is outside the band
    for a in range(3):
        for s in (-1, 1):
            NK = K.copy()
            NK[:, a] += s
            absent = ix.pde(NK) < 0
            Y = NK[absent] / float(N)
            E = Y - S.cp(Y)
            dd = np.sqrt((E[:, 0] * E[:, 0] + E[:, 1] * E[:, 1]) + E[:, 2] * E[:, 2])
            assert np.all(~(dd <= r))
    # tube volume
    if isinstance(S, G.Sphere):
        vol = 4 * np.pi / 3 * ((1 + r) ** 3 - (1 - r) ** 3)
    else:
        vol = 8 * np.pi ** 2 * S.R * S.rho * r
    assert abs(band.n_s - vol * N ** 3) / band.n_s < 0.005


@pytest.mark.parametrize("name", ["sphere_lat_256", "torus_meridians_512"])
def test_fullsize_apply_sampled_rows(name):
    import torch
    from paper_2305_04711_amd import cpm
    S, Cs, N, band, ix, loc = _setup(name)
    rng = np.random.default_rng(21)
    u_np = rng.standard_normal(band.n)
    Ks, curve, gpu_rows = _samples(S, Cs, N, band, ix, rng)
    m, n = 0.25, -1.0

    def u_of(K, c):
        return u_np[ix.dof(K, c)]

    ref = loc.apply_rows(Ks, curve, u_of, m, n)
    scale = np.max(np.abs(ref))
    for td, tol in ((torch.float64, 1e-12), (torch.float32, 5e-6)):
        u = torch.tensor(u_np, dtype=td, device="cuda")
        v = cpm.apply(band, u, m, n).cpu().numpy().astype(np.float64)
        err = np.max(np.abs(v[gpu_rows] - ref)) / scale
        print(name, td, "sampled rows", gpu_rows.size, "rel err", err, flush=True)
        assert err < tol


@pytest.mark.parametrize("name", ["sphere_lat_256", "torus_meridians_512"])
def test_fullsize_apply_every_launch_variant(name):
    """Each of the launch variants (LDS padding x tile order, including the
    persistent gather, whose wavefronts each take many tiles here, x the two
    forms of the Laplacian pass) on the sampled rows; the autotuned choice is
    restored afterwards."""
    import torch
    from paper_2305_04711_amd import cpm
    S, Cs, N, band, ix, loc = _setup(name)
    rng = np.random.default_rng(23)
    u_np = rng.standard_normal(band.n)
    Ks, curve, gpu_rows = _samples(S, Cs, N, band, ix, rng)
    m, n = 0.0, -1.0

    def u_of(K, c):
        return u_np[ix.dof(K, c)]

    ref = loc.apply_rows(Ks, curve, u_of, m, n)
    scale = np.max(np.abs(ref))
    try:
        for td, tol in ((torch.float64, 1e-12), (torch.float32, 5e-6)):
            u = torch.tensor(u_np, dtype=td, device="cuda")
            for k in range(capi.TUNE_VARIANTS):
                cpm.tune_set(band, td, k)
                v = cpm.apply(band, u, m, n).cpu().numpy().astype(np.float64)
                err = np.max(np.abs(v[gpu_rows] - ref)) / scale
                print(name, td, "variant", k, "rel err", err, flush=True)
                assert err < tol
    finally:
        cpm.autotune(band, torch.float64)
        cpm.autotune(band, torch.float32)


def test_fullsize_sphere_latitude_solve():
    import torch
    from paper_2305_04711_amd import cpm
    S, Cs, N, band, ix, loc = _setup("sphere_lat_256")
    cpc = band.bc_cpc()
    g = torch.tensor(np.sin(2 * np.arctan2(cpc[:, 1], cpc[:, 0])), device="cuda")
    f = torch.zeros(band.n_s, dtype=torch.float64, device="cuda")
    b = cpm.rhs(band, f, g, -1.0)
    x, st = cpm.solve(band, b, 0.0, -1.0, tol=1e-10, mode="mixed")
    print("C3 solve", st, flush=True)
    assert st["converged"] and st["relres"] <= 1e-10
    xn = x.cpu().numpy()
    bn = b.cpu().numpy()
    rng = np.random.default_rng(22)
    Ks, curve, gpu_rows = _samples(S, Cs, N, band, ix, rng)

    def u_of(K, c):
        return xn[ix.dof(K, c)]

    Ax = loc.apply_rows(Ks, curve, u_of, 0.0, -1.0)
    res = np.abs(bn[gpu_rows] - Ax)
    # relres 1e-10 in the 2-norm bounds every entry of the residual
    assert np.max(res) <= 1e-10 * np.linalg.norm(bn) * 1.0001
    # surface values E u against the stereographic closed form (2nd order)
    pde = curve < 0
    sv = loc._E_pde(Ks[pde], u_of)
    err = np.max(np.abs(sv - latitude_harmonic(band.cp()[gpu_rows[pde]], 0.3)))
    print("C3 closed-form Linf on sampled rows", err, flush=True)
    # the oracle's errors at h = 1/16 .. 1/48 (3.2e-3 .. 3.9e-4) extrapolate
    # to about 2e-5 at h = 1/256
    assert err < 4e-5


@pytest.mark.parametrize("mode", ["mixed", "f64"])
def test_fullsize_torus_solve_in_the_bench_configuration(mode):
    """The solve bench.py times (torus h = 1/512, meridian Dirichlet IBCs,
    the bench's seeded f and g, Poisson, tol 1e-8): the residual of sampled
    rows, evaluated by the oracle row by row from the GPU solution, is
    bounded by the 2-norm relative residual the solver reports."""
    import torch
    from paper_2305_04711_amd import cpm
    S, Cs, N, band, ix, loc = _setup("torus_meridians_512")
    cp = band.cp()
    f = torch.tensor(inputs.torus_field(inputs.torus_coeffs(100), cp), device="cuda")
    g = torch.tensor(inputs.meridian_dirichlet(band.bc_cpc(), seed=2), device="cuda")
    b = cpm.rhs(band, f, g, -1.0)
    x, st = cpm.solve(band, b, 0.0, -1.0, tol=1e-8, mode=mode)
    print("C5 solve", mode, st, flush=True)
    assert st["converged"] and st["relres"] <= 1e-8
    xn = x.cpu().numpy()
    bn = b.cpu().numpy()
    rng = np.random.default_rng(24)
    Ks, curve, gpu_rows = _samples(S, Cs, N, band, ix, rng)

    def u_of(K, c):
        return xn[ix.dof(K, c)]

    Ax = loc.apply_rows(Ks, curve, u_of, 0.0, -1.0)
    res = np.abs(bn[gpu_rows] - Ax)
    assert np.max(res) <= 1e-8 * np.linalg.norm(bn) * 1.0001


def test_largest_size_apply_sampled_rows():
    """The torus with meridian IBCs at h = 1/1024: about 137M DOFs (the band is
    a shell, so DOFs grow as N^2), 4x the bench workload.  Sampled rows
    against the oracle's row-by-row evaluation, FP64 and FP32."""
    import torch
    from paper_2305_04711_amd import cpm
    S, Cs, N, band, ix, loc = _setup("torus_meridians_1024")
    assert band.n > 1.3e8
    rng = np.random.default_rng(25)
    Ks, curve, gpu_rows = _samples(S, Cs, N, band, ix, rng)
    u_np = rng.standard_normal(band.n)
    m, n = 0.0, -1.0

    def u_of(K, c):
        return u_np[ix.dof(K, c)]

    ref = loc.apply_rows(Ks, curve, u_of, m, n)
    scale = np.max(np.abs(ref))
    for td, tol in ((torch.float64, 1e-12), (torch.float32, 5e-6)):
        u = torch.tensor(u_np, dtype=td, device="cuda")
        v = cpm.apply(band, u, m, n)
        vr = v[torch.tensor(gpu_rows, device="cuda")].cpu().numpy().astype(np.float64)
        del u, v
        err = np.max(np.abs(vr - ref)) / scale
        print("h=1/1024", td, "sampled rows", gpu_rows.size, "rel err", err, flush=True)
        assert err < tol
    _cache.pop("torus_meridians_1024", None)


def test_index_range_limit_fails_cleanly():
    """A band past the 32-bit DOF range (torus at h = 1/4096, about 2.2G
    nodes) is refused with CPM_E_INVALID before its arrays are built."""
    from paper_2305_04711_amd import capi, cpm
    with pytest.raises(capi.CPMError) as ei:
        cpm.Band(cpm.torus(1.0, 0.4), [], 4096)
    assert ei.value.status == capi.E_INVALID
    assert "too large" in str(ei.value) or "index range" in str(ei.value)

