"""Time stepping of the heat equation u_t = Delta_S u with interior boundary
conditions (the paper's heat test, Sec. 6.2): Crank-Nicolson (trapezoidal
rule) in time on the CPM system of Sec. 5.4.

With M the linear part of the stabilised operator diag(L) + (L - diag L) E
and e(g) the Dirichlet constants of E, the semi-discrete system is
u' = M u + (L - diag L) e(g(t)), and one trapezoidal step reads

    (I - dt/2 M) u^{k+1} = (I + dt/2 M) u^k + dt/2 (L - diag L) (e(g^k) + e(g^{k+1})).

Test infrastructure only.  Each step is solved with the oracle's BiCGSTAB
(I - dt/2 M is well conditioned for dt ~ h) to a relative residual of tol.
"""

import numpy as np
import scipy.sparse as sp

from .krylov import bicgstab


def heat_cn(sysm, u0, dt, nsteps, g_steps=None, tol=1e-13):
    """u^nsteps from u^0 by nsteps Crank-Nicolson steps of size dt.
    g_steps: (nsteps + 1, n_c) Dirichlet data at t_k = k dt (None: no BC DOFs
    or no Dirichlet side).  Returns the final state (n,)."""
    n = sysm.n
    M = (sp.diags(sysm.diagL) + sysm.L_off @ sysm.E).tocsr()
    u = np.asarray(u0, dtype=np.float64).copy()
    for k in range(nsteps):
        b = u + 0.5 * dt * (M @ u)
        if g_steps is not None and sysm.n_c:
            e = sysm.e_vector(g_steps[k]) + sysm.e_vector(g_steps[k + 1])
            b = b + 0.5 * dt * (sysm.L_off @ e)
        u, info = bicgstab(lambda x: x - 0.5 * dt * (M @ x), b, x0=u, tol=tol)
        if not info["converged"]:
            raise RuntimeError("Crank-Nicolson step %d did not converge: %s" % (k, info))
    return u
