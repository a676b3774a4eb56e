"""Pins of the oracle's stencil-set band (Sec. 5.1 cites the construction:
only the grid points that interpolation and FD stencils need)."""

import itertools

import numpy as np
import pytest
import scipy.sparse.linalg as spl

from oracle import geometry as G
from oracle import operator as O
from oracle.band import node_coords



def _config(name):
    if name == "circle_point":
        S = G.Circle()
        return S, [G.PointC((1.0, 0.0), (0.0, 1.0))], None, (0.0, -1.0)
    if name == "sphere_lat":
        S = G.Sphere()
        return S, [G.LatitudeC(S, 0.3)], None, (0.0, -1.0)
    if name == "torus_meridians":
        S = G.Torus(1.0, 0.4)
        return S, [G.MeridianC(S, 1.0, 0.0), G.MeridianC(S, -1.0, 0.0)], None, (0.0, -1.0)
    S = G.Sphere()
    return S, [G.LatitudeC(S, 0.0)], [("neumann", "neumann")], (1.0, -1.0)


@pytest.mark.parametrize("name,N,p", [("circle_point", 32, 3), ("sphere_lat", 16, 3),
                                      ("torus_meridians", 12, 3), ("sphere_eq_neumann", 14, 3),
                                      ("sphere_lat", 16, 2)])
def test_stencil_set_keeps_the_surface_solution(name, N, p):
    """The rows of every stencil-referenced DOF are those of the tube system,
    so the interpolated surface values E u agree at every node of the smaller
    band, with the same f and g (a dropped row or a wrong index would move
    them at O(1))."""
    S, Cs, bct, (m, n) = _config(name)
    T = O.CPMSystem(S, N, Cs, bc_types=bct, p=p)
    Q = O.CPMSystem(S, N, Cs, bc_types=bct, p=p, band="stencil_set")
    assert Q.n < T.n
    rng = np.random.default_rng(5)
    fT = rng.standard_normal(T.n_s)
    gT = rng.standard_normal(T.n_c)
    iT = T.index(Q.K)
    assert np.all(iT >= 0)
    fQ = fT[iT]
    gQ = np.array([gT[T.alpha_of[c][iT[j]] - T.n_s] for c, j in zip(Q.bc_curve, Q.bc_node)])
    xT = spl.spsolve(T.matrix(m, n).tocsc(), T.rhs(fT, gT, n))
    xQ = spl.spsolve(Q.matrix(m, n).tocsc(), Q.rhs(fQ, gQ, n))
    sT = T.surface_values(xT, gT)[iT]
    sQ = Q.surface_values(xQ, gQ)
    assert np.max(np.abs(sT - sQ)) <= 1e-10 * np.max(np.abs(sT))


@pytest.mark.parametrize("N,p", [(32, 3), (64, 3), (32, 2)])
def test_stencil_set_reduction_on_the_unit_sphere(N, p):
    """Sec. 5.1 quotes 6-15% fewer DOFs for the unit sphere."""
    T = O.CPMSystem(G.Sphere(), N, p=p)
    keep = O.stencil_set_nodes(T)
    red = 1.0 - keep.sum() / T.n_s
    assert 0.06 <= red <= 0.15, red


def test_stencil_set_against_brute_force_geometry():
    """Without interior boundaries the set is: every member of the cubic
    stencil of cp_S(x) for every tube node x, and their face neighbours that
    are tube nodes, found here from the coordinates alone."""
    S, N = G.Circle(), 24
    T = O.CPMSystem(S, N)
    tube = set(map(tuple, T.K.tolist()))
    members = set()
    for k, y in zip(T.K.tolist(), T.CP.tolist()):
        b = [int(np.floor(c * N)) - 1 for c in y]
        for off in itertools.product(range(4), repeat=2):
            members.add((b[0] + off[0], b[1] + off[1]))
    assert members <= tube
    need = set(members)
    for (i, j) in members:
        for di, dj in ((1, 0), (-1, 0), (0, 1), (0, -1)):
            if (i + di, j + dj) in tube:
                need.add((i + di, j + dj))
    keep = O.stencil_set_nodes(T)
    got = set(map(tuple, T.K[keep].tolist()))
    assert got == need
    # and the stencil-set system is built on exactly these nodes
    Q = O.CPMSystem(S, N, band="stencil_set")
    assert set(map(tuple, Q.K.tolist())) == need
    assert np.array_equal(node_coords(Q.K, N).shape, (len(need), 2))
