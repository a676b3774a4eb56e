"""Mapping between the HIP library's DOF order (block order) and the oracle's
(lexicographic) through exported grid coordinates, and the configurations
shared by the GPU parity tests."""

import numpy as np

from oracle import geometry as G
from oracle import operator as O


def oracle_and_gpu(cfg, N, order=2, degree=3, band="tube"):
    """Build the oracle system and the GPU band for a named configuration
    (interpolation degree: 3 cubic, 2 quadratic; band: "tube" or
    "stencil_set")."""
    from paper_2305_04711_amd import cpm
    if cfg == "circle_point":
        S = G.Circle()
        Cs = [G.PointC((1.0, 0.0), (0.0, 1.0))]
        gs, gi = cpm.circle(), [cpm.point_ibc((1.0, 0.0), (0.0, 1.0))]
    elif cfg == "circle_jump":
        thc = 1.022 * np.pi
        p = (np.cos(thc), np.sin(thc))
        S = G.Circle()
        Cs = [G.PointC(p, (-p[1], p[0]))]
        gs, gi = cpm.circle(), [cpm.point_ibc(p, (-p[1], p[0]))]
    elif cfg == "sphere":
        S, Cs = G.Sphere(), []
        gs, gi = cpm.sphere(), []
    elif cfg == "sphere_lat":
        S = G.Sphere()
        Cs = [G.LatitudeC(S, 0.3)]
        gs, gi = cpm.sphere(), [cpm.latitude_ibc(0.3)]
    elif cfg == "torus":
        S, Cs = G.Torus(1.0, 0.4), []
        gs, gi = cpm.torus(1.0, 0.4), []
    elif cfg == "torus_meridians":
        S = G.Torus(1.0, 0.4)
        Cs = [G.MeridianC(S, 1.0, 0.0), G.MeridianC(S, -1.0, 0.0)]
        gs, gi = cpm.torus(1.0, 0.4), [cpm.meridian_ibc(1.0, 0.0), cpm.meridian_ibc(-1.0, 0.0)]
    elif cfg == "sphere_point":
        a, b = 1.1, 0.7
        pt = (np.sin(a) * np.cos(b), np.sin(a) * np.sin(b), np.cos(a))
        o = (np.cos(a) * np.cos(b), np.cos(a) * np.sin(b), -np.sin(a))
        S = G.Sphere()
        Cs = [G.PointC(pt, o)]
        gs, gi = cpm.sphere(), [cpm.point_ibc(pt, o)]
    elif cfg in ("sphere_arc", "sphere_arc_neumann"):
        if cfg == "sphere_arc":
            z0, a0, a1, bct = 0.3, -0.75 * np.pi, 0.25 * np.pi, [("dirichlet", "dirichlet")]
        else:
            z0, a0, a1, bct = 0.0, 0.3, 0.3 + 1.4 * np.pi, [("neumann", "neumann")]
        a, b = (np.cos(a0), np.sin(a0)), (np.cos(a1), np.sin(a1))
        S = G.Sphere()
        Cs = [G.LatitudeArc(S, z0, a, b)]
        gs, gi = cpm.sphere(), [cpm.latitude_arc_ibc(z0, a, b, bc=bct[0])]
    elif cfg == "sphere_eq_neumann":
        S = G.Sphere()
        Cs, bct = [G.LatitudeC(S, 0.0)], [("neumann", "neumann")]
        gs, gi = cpm.sphere(), [cpm.latitude_ibc(0.0, bc="neumann")]
    elif cfg == "sphere_eq_mixed":
        S = G.Sphere()
        Cs, bct = [G.LatitudeC(S, 0.0)], [("dirichlet", "neumann")]
        gs, gi = cpm.sphere(), [cpm.latitude_ibc(0.0, bc=("dirichlet", "neumann"))]
    elif cfg == "circle_mixed":
        S = G.Circle()
        Cs, bct = [G.PointC((1.0, 0.0), (0.0, 1.0))], [("neumann", "dirichlet")]
        ib = cpm.point_ibc((1.0, 0.0), (0.0, 1.0))
        ib.bc[0], ib.bc[1] = 1, 0
        gs, gi = cpm.circle(), [ib]
    else:
        raise KeyError(cfg)
    bc_types = bct if cfg in NEUMANN_CASES or cfg == "sphere_arc" else None
    sysm = O.CPMSystem(S, N, Cs, order=order, bc_types=bc_types, p=degree, band=band)
    gband = cpm.Band(gs, gi, N, order=order, p=degree, band=band)
    return sysm, gband


# configurations with a zero-Neumann side (screened operators: m = 1)
NEUMANN_CASES = ("sphere_eq_neumann", "sphere_eq_mixed", "circle_mixed", "sphere_arc_neumann")


def dof_map(sysm, band):
    """g2o[i] = oracle DOF of GPU DOF i (PDE and BC)."""
    K = band.coords().astype(np.int64)
    pde = sysm.index(K)
    assert np.all(pde >= 0), "GPU band node missing from the oracle band"
    g2o = np.empty(band.n, dtype=np.int64)
    g2o[:band.n_s] = pde
    if band.n_c:
        node = band.bc_node()
        curve = band.bc_curve()
        onode = pde[node]
        bc = np.array([sysm.alpha_of[c][j] for c, j in zip(curve, onode)], dtype=np.int64)
        assert np.all(bc >= 0), "GPU BC DOF at a node without an oracle BC DOF"
        g2o[band.n_s:] = bc
    assert np.unique(g2o).size == band.n
    return g2o


def to_gpu_order(x_oracle, g2o):
    return np.asarray(x_oracle)[..., g2o]
