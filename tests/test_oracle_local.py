"""Pins the oracle's row-by-row evaluator (used for sampled checks at full
size) to the assembled oracle system: every row agrees with CPMSystem.apply."""

import numpy as np
import pytest

from oracle import geometry as G
from oracle import local as LO
from oracle import operator as O


def _u_of_factory(sysm, u):
    def u_of(K, curve):
        pde = sysm.index(K)
        assert np.all(pde >= 0)
        out = u[pde].copy()
        for ci in range(len(sysm.alpha_of)):
            m = curve == ci
            if m.any():
                a = sysm.alpha_of[ci][pde[m]]
                assert np.all(a >= 0)
                out[m] = u[a]
        return out
    return u_of


def _cases():
    T = G.Torus(1.0, 0.4)
    S = G.Sphere()
    p = (np.cos(1.022 * np.pi), np.sin(1.022 * np.pi))
    return [
        ("circle_point", G.Circle(), [G.PointC((1.0, 0.0), (0.0, 1.0))], 32, 2),
        ("circle_jump_o1", G.Circle(), [G.PointC(p, (-p[1], p[0]))], 48, 1),
        ("sphere", S, [], 10, 2),
        ("sphere_lat", S, [G.LatitudeC(S, 0.3)], 14, 2),
        ("torus_meridians", T, [G.MeridianC(T, 1.0, 0.0), G.MeridianC(T, -1.0, 0.0)], 12, 2),
    ]


@pytest.mark.parametrize("name,S,Cs,N,order", _cases())
def test_local_rows_equal_assembled_operator(name, S, Cs, N, order):
    sysm = O.CPMSystem(S, N, Cs, order=order)
    u = np.random.default_rng(3).standard_normal(sysm.n)
    m, n = 0.3, -1.1
    ref = sysm.apply(u, m, n)
    loc = LO.LocalCPM(S, N, Cs, order=order)
    K = np.concatenate([sysm.K, sysm.K[sysm.bc_node]])
    curve = np.concatenate([np.full(sysm.n_s, -1), sysm.bc_curve])
    got = loc.apply_rows(K, curve, _u_of_factory(sysm, u), m, n)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref)), name


def test_local_rows_refuse_what_they_do_not_model():
    S = G.Sphere()
    arc = G.LatitudeArc(S, 0.3, (1.0, 0.0), (0.0, 1.0))
    with pytest.raises(NotImplementedError):
        LO.LocalCPM(S, 16, [arc])
    with pytest.raises(NotImplementedError):
        LO.LocalCPM(S, 16, [G.LatitudeC(S, 0.0)], bc_types=[("neumann", "neumann")])
    with pytest.raises(NotImplementedError):
        LO.LocalCPM(S, 16, [], p=2)
    with pytest.raises(NotImplementedError):
        LO.LocalCPM(S, 16, [], band="stencil_set")
    with pytest.raises(NotImplementedError):
        LO.LocalCPM(S, 16, [G.LatitudeC(S, 0.3)], order=3)
