"""Writes tests/golden/adjoint_torus128.npz with the oracle only.

Differentiable solve on the torus R = 1, rho = 0.4 at h = 1/128 with two
second-order Dirichlet meridians (toroidal angles 0 and pi): Poisson
(m = 0, n = -1),
    u = A^-1 b(f, g),  loss = sum_{PDE DOFs} (u - t)^2,
f = seeded torus modes (seed 100), g = meridian data (seed 2), t = seeded torus
modes (seed 3), all evaluated at the closest points.  Stores the loss, the
gradient with respect to every Dirichlet value (keyed by node coordinates
and curve) and to f at 4000 seeded nodes, and the solution there.

Run from the repository root:  python tests/golden/make_adjoint_golden.py
"""

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import adjoint as AD  # noqa: E402
from oracle import geometry as G  # noqa: E402
from oracle import krylov as KR  # noqa: E402
from oracle import operator as O  # noqa: E402
from paper_2305_04711_amd import inputs  # noqa: E402

N = int(os.environ.get("GOLDEN_N", "128"))


def main():
    t0 = time.time()
    T = G.Torus(1.0, 0.4)
    sysm = O.CPMSystem(T, N, [G.MeridianC(T, 1.0, 0.0), G.MeridianC(T, -1.0, 0.0)])
    print("system", sysm.n_s, sysm.n_c, "%.0fs" % (time.time() - t0), flush=True)
    m, n = 0.0, -1.0
    f = inputs.torus_field(inputs.torus_coeffs(100), sysm.CP)
    g = inputs.meridian_dirichlet(sysm.bc_cpc, seed=2)
    tgt = inputs.torus_field(inputs.torus_coeffs(3), sysm.CP)
    b = sysm.rhs(f, g, n)
    u, info = KR.bicgstab(lambda x: sysm.apply(x, m, n), b, tol=1e-12)
    print("forward", info, "%.0fs" % (time.time() - t0), flush=True)
    loss = AD.loss(sysm, u, tgt)
    lam, info2 = AD.solve_adjoint(sysm, AD.adjoint_rhs(sysm, u, tgt), m, n, tol=1e-12)
    print("adjoint", info2, "%.0fs" % (time.time() - t0), flush=True)
    gf, gg = AD.rhs_gradients(sysm, lam, n)
    rng = np.random.default_rng(5)
    pick = np.sort(rng.choice(sysm.n_s, 4000, replace=False))
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "adjoint_torus%d.npz" % N)
    np.savez_compressed(out, N=N, loss=loss, relres_forward=info["relres"],
                        relres_adjoint=info2["relres"],
                        bc_coords=sysm.K[sysm.bc_node].astype(np.int32),
                        bc_curve=sysm.bc_curve.astype(np.int32), grad_g=gg,
                        f_coords=sysm.K[pick].astype(np.int32), grad_f=gf[pick],
                        u=u[pick])
    print("wrote", out, "%.0fs" % (time.time() - t0), flush=True)


if __name__ == "__main__":
    main()
