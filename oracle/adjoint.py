"""Adjoint of the CPM solve (not in the paper; derived from the system of
Sec. 5.4).

Forward:  A u = b(f, g),  A = m I + n [diag L + L_off E],
          b = P f - n L_off e(g),  e(g) = c_ord g on BC DOFs (c_ord = 1 or 2),
          P f copies f to the BC DOF of the same node.
Loss:     l(u) = sum_{i in J_S} (u_i - t_i)^2  (PDE DOFs only).
Adjoint:  A^T lam = dl/du = [2 (u - t) on J_S; 0 on J_C]
          A^T = m I + n [diag L + E^T L_off^T]  (transposes of the CSR)
Gradients: dl/df_j = lam_j + sum_{alpha on node j} lam_alpha
           dl/dg   = -n c_ord (L_off^T lam) restricted to J_C
"""

import numpy as np

from .krylov import bicgstab


def apply_transpose(sysm, w, m, n):
    """A^T w from the transposed CSR factors, in the order the transpose of
    the four-step product takes: c = L_off^T w, then E^T c."""
    c = sysm.L_off.T @ w
    return m * w + n * (sysm.diagL * w) + n * (sysm.E.T @ c)


def loss(sysm, u, target):
    d = u[:sysm.n_s] - target
    return float(np.dot(d, d))


def adjoint_rhs(sysm, u, target):
    r = np.zeros(sysm.n)
    r[:sysm.n_s] = 2.0 * (u[:sysm.n_s] - target)
    return r


def rhs_gradients(sysm, lam, n):
    """(grad_f, grad_g) of l through b(f, g) given the adjoint state lam."""
    grad_f = lam[:sysm.n_s].copy()
    np.add.at(grad_f, sysm.bc_node, lam[sysm.n_s:])
    c = sysm.L_off.T @ lam
    grad_g = -n * sysm.e_coef * c[sysm.n_s:]
    return grad_f, grad_g


def solve_adjoint(sysm, rhs, m, n, tol=1e-12, dense=False):
    if dense:
        At = sysm.matrix(m, n).T.toarray()
        return np.linalg.solve(At, rhs), dict(iters=0, relres=0.0, converged=True)
    return bicgstab(lambda w: apply_transpose(sysm, w, m, n), rhs, tol=tol)
