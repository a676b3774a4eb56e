"""Pins of the oracle's closest-point functions and band construction against
identities, brute force and analytic volumes (CPU only)."""

import numpy as np
import pytest

from oracle import band as B
from oracle import geometry as G
from oracle import operator as O


def _pts(n, dim, scale, seed):
    return np.random.default_rng(seed).uniform(-scale, scale, (n, dim))


def test_band_radius_factor_matches_eq_bandwidth():
    # eq. (bandwidth) with p = 3, q = 1
    assert G.band_radius_factor(2) == 13.0
    assert G.band_radius_factor(3) == 17.0
    # p = 2: (d-1) 2.25 + 2.5^2
    assert G.band_radius_factor(3, p=2) == pytest.approx(10.75)


@pytest.mark.parametrize("S", [G.Circle(1.0, (0.1, -0.2)), G.Sphere(1.3, (0.1, 0.2, -0.3))])
def test_cp_round_objects(S):
    X = _pts(2000, S.dim, 2.0, 1)
    CP = S.cp(X)
    d = CP - S.c
    assert np.allclose(np.sqrt(np.sum(d * d, axis=1)), S.R, atol=1e-14)
    assert np.allclose(S.cp(CP), CP, atol=1e-14)             # idempotent
    # x - c and cp - c point the same way
    u = (X - S.c) / np.linalg.norm(X - S.c, axis=1)[:, None]
    assert np.allclose(u * S.R, d, atol=1e-14)


def test_cp_torus_brute_force():
    T = G.Torus(1.0, 0.4)
    X = _pts(300, 3, 1.3, 2)
    X = X[np.abs(np.sqrt(X[:, 0] ** 2 + X[:, 1] ** 2) - 1.0) < 0.35]
    CP = T.cp(X)
    # on the torus
    rr = np.sqrt(CP[:, 0] ** 2 + CP[:, 1] ** 2)
    assert np.allclose((rr - 1.0) ** 2 + CP[:, 2] ** 2, 0.16, atol=1e-13)
    assert np.allclose(T.cp(CP), CP, atol=1e-13)
    # brute force over a fine parameter grid
    ph, th = np.meshgrid(np.linspace(0, 2 * np.pi, 1200, endpoint=False),
                         np.linspace(0, 2 * np.pi, 600, endpoint=False), indexing="ij")
    P = np.stack([(1 + 0.4 * np.cos(th)) * np.cos(ph), (1 + 0.4 * np.cos(th)) * np.sin(ph),
                  0.4 * np.sin(th)], axis=-1).reshape(-1, 3)
    for x, c in zip(X[:40], CP[:40]):
        dmin = np.min(np.linalg.norm(P - x, axis=1))
        assert np.linalg.norm(c - x) <= dmin + 1e-12
        assert np.linalg.norm(c - x) >= dmin - 6e-3


def test_cp_curves_brute_force():
    S = G.Sphere()
    lat = G.LatitudeC(S, 0.3)
    T = G.Torus(1.0, 0.4)
    mer = G.MeridianC(T, -1.0, 0.0)
    X = _pts(60, 3, 1.2, 3)
    s = np.linspace(0, 2 * np.pi, 20000, endpoint=False)
    rho0 = np.sqrt(1 - 0.09)
    P_lat = np.stack([rho0 * np.cos(s), rho0 * np.sin(s), np.full_like(s, 0.3)], axis=1)
    P_mer = np.stack([-1.0 - 0.4 * np.cos(s), np.zeros_like(s), 0.4 * np.sin(s)], axis=1)
    for curve, P in ((lat, P_lat), (mer, P_mer)):
        CPC = curve.cp(X)
        for x, c in zip(X, CPC):
            dmin = np.min(np.linalg.norm(P - x, axis=1))
            assert abs(np.linalg.norm(c - x) - dmin) < 1e-6
    # orientation vectors: unit, tangent to S, normal to C
    o = lat.orient(lat.cp(X))
    assert np.allclose(np.linalg.norm(o, axis=1), 1.0)
    cpc = lat.cp(X)
    assert np.allclose(np.sum(o * cpc, axis=1), 0.0, atol=1e-14)   # tangent to sphere
    assert np.all(o[:, 2] > 0)                                        # north
    assert np.allclose(mer.orient(X), [0.0, -1.0, 0.0])


@pytest.mark.parametrize("S,N", [(G.Circle(), 32), (G.Sphere(), 8), (G.Torus(1.0, 0.4), 10)])
def test_scan_equals_bfs_algorithm1(S, N):
    K, _ = B.scan_band(S, N)
    got = B.bfs_band(S, N, K[len(K) // 2])
    assert got == set(map(tuple, K.tolist()))


def test_band_counts_match_tube_volume():
    # circle: area of the annulus 4 pi r, / h^2
    K, _ = B.scan_band(G.Circle(), 32)
    r = np.sqrt(13) / 32
    assert abs(len(K) - 4 * np.pi * r * 32 ** 2) / len(K) < 0.01
    # sphere: (4 pi / 3)((1 + r)^3 - (1 - r)^3) / h^3
    for N in (24, 48):
        K, _ = B.scan_band(G.Sphere(), N)
        r = np.sqrt(17) / N
        vol = 4 * np.pi / 3 * ((1 + r) ** 3 - (1 - r) ** 3)
        assert abs(len(K) - vol * N ** 3) / len(K) < 0.01
    # torus: 8 pi^2 R rho r / h^3
    K, _ = B.scan_band(G.Torus(1.0, 0.4), 32)
    r = np.sqrt(17) / 32
    assert abs(len(K) - 8 * np.pi ** 2 * 0.4 * r * 32 ** 3) / len(K) < 0.01


def test_band_membership_is_the_definition():
    S = G.Sphere()
    N = 12
    K, CP = B.scan_band(S, N)
    X = K / N
    d = np.sqrt(np.sum((X - CP) ** 2, axis=1))
    assert np.all(d <= np.sqrt(17) / N)
    # every node outside the set (in the box) fails the test
    lo, hi = K.min(0) - 2, K.max(0) + 2
    g = np.stack(np.meshgrid(*[np.arange(a, b + 1) for a, b in zip(lo, hi)],
                             indexing="ij"), -1).reshape(-1, 3)
    Xg = g / N
    dg = np.linalg.norm(Xg - S.cp(Xg), axis=1)
    inside = set(map(tuple, g[dg <= np.sqrt(17) / N].tolist()))
    assert inside == set(map(tuple, K.tolist()))


def test_narrow_band_leaves_stencil_holes():
    # a 2.5h band cannot hold the 4^d cubic stencils
    with pytest.raises(O.StencilHole):
        O.CPMSystem(G.Circle(), 32, r=2.5 / 32)
    with pytest.raises(O.StencilHole):
        O.CPMSystem(G.Sphere(), 16, r=2.5 / 16)


def test_omega_c_and_check_region_are_the_definitions():
    S = G.Circle()
    C = G.PointC((1.0, 0.0), (0.0, 1.0))
    sysm = O.CPMSystem(S, 32, [C])
    X = sysm.K / 32
    d = np.linalg.norm(X - np.array([1.0, 0.0]), axis=1)
    r = np.sqrt(13) / 32
    assert np.array_equal(np.nonzero(d <= r)[0], sysm.bc_node)
    assert np.array_equal(sysm.sets[0].in_check, d < 2 * r)
    assert sysm.n_c == int(np.sum(d <= r))
    # BC DOFs are numbered after the PDE DOFs (Sec. 4.1)
    assert sysm.n == sysm.n_s + sysm.n_c


@pytest.mark.parametrize("a_ang,b_ang", [(-0.75 * np.pi, 0.25 * np.pi), (0.3, 0.3 + 1.4 * np.pi)])
def test_latitude_arc_cp_and_boundary_brute_force(a_ang, b_ang):
    """cp_C of an open arc (Sec. 4.4) is the nearest arc point (brute force
    over a fine sampling of the arc, half-turn and longer arcs) and Omega(dC)
    (eq. IBC_boundary_set) is exactly where the nearest arc point is an
    endpoint."""
    S = G.Sphere()
    z0 = 0.3
    arc = G.LatitudeArc(S, z0, (np.cos(a_ang), np.sin(a_ang)), (np.cos(b_ang), np.sin(b_ang)))
    rho0 = np.sqrt(1 - z0 * z0)
    span = (b_ang - a_ang) % (2 * np.pi)
    t = a_ang + span * np.linspace(0.0, 1.0, 20001)
    P = np.stack([rho0 * np.cos(t), rho0 * np.sin(t), np.full(t.size, z0)], axis=1)
    X = _pts(400, 3, 1.3, 11)
    X = X[np.abs(np.linalg.norm(X, axis=1) - 1.0) < 0.3]
    CP = arc.cp(X)
    end = arc.at_boundary(X)
    for x, c, e in zip(X, CP, end):
        d = np.linalg.norm(P - x, axis=1)
        k = int(np.argmin(d))
        assert np.linalg.norm(c - x) <= d[k] + 1e-12
        assert np.linalg.norm(c - x) >= d[k] - 2e-4
        if k not in (0, t.size - 1) and d[k] < min(d[0], d[-1]) - 1e-3:
            assert not e
        if k in (0, t.size - 1) and d[k] < np.min(d[1:-1]) - 1e-9:
            assert e
    assert end.any() and (~end).any()
