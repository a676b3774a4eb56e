"""Linear solvers for the oracle, FP64 throughout.

* ``dense_solve``: assemble A densely and solve by LU (numpy.linalg.solve,
  i.e. LAPACK getrf/getrs) - the brute-force reference on tiny grids.
* ``bicgstab``: unpreconditioned BiCGSTAB of van der Vorst (1992), the method
  the paper's solver follows (Sec. 5.4).  With a scalar diagonal
  preconditioner it is unchanged up to scaling, since diag(m I + n diag L) is
  a constant on a uniform grid.
* ``gmres``: restarted GMRES(k) with modified Gram-Schmidt and Givens
  rotations (Saad and Schultz 1986).

All stop when ||b - A x||_2 <= tol ||b||_2 (relative residual), measured on
the true residual at exit.
"""

import numpy as np


def dense_solve(A, b):
    Ad = A.toarray() if hasattr(A, "toarray") else np.asarray(A)
    return np.linalg.solve(Ad, b)


def bicgstab(matvec, b, x0=None, tol=1e-12, maxiter=100000):
    """Returns (x, info) with info = dict(iters, relres, converged)."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    bn = np.linalg.norm(b)
    if bn == 0.0:
        return np.zeros_like(b), dict(iters=0, relres=0.0, converged=True)
    r = b - matvec(x)
    rhat = r.copy()
    rho_old = alpha = omega = 1.0
    v = np.zeros_like(b)
    p = np.zeros_like(b)
    it = 0
    restarts = 0
    while it < maxiter:
        rho = np.dot(rhat, r)
        if abs(rho) < 1e-300 or omega == 0.0:
            # breakdown: restart from the current iterate with a new shadow
            r = b - matvec(x)
            rhat = r.copy()
            rho_old = alpha = omega = 1.0
            v[:] = 0.0
            p[:] = 0.0
            restarts += 1
            if restarts > 50:
                break
            continue
        beta = (rho / rho_old) * (alpha / omega)
        p = r + beta * (p - omega * v)
        v = matvec(p)
        alpha = rho / np.dot(rhat, v)
        s = r - alpha * v
        if np.linalg.norm(s) <= tol * bn:
            x = x + alpha * p
            it += 1
            break
        t = matvec(s)
        tt = np.dot(t, t)
        omega = np.dot(t, s) / tt if tt > 0.0 else 0.0
        x = x + alpha * p + omega * s
        r = s - omega * t
        rho_old = rho
        it += 1
        if np.linalg.norm(r) <= tol * bn:
            # confirm on the true residual
            rt = b - matvec(x)
            if np.linalg.norm(rt) <= tol * bn:
                break
            r = rt
            rhat = r.copy()
            rho_old = alpha = omega = 1.0
            v[:] = 0.0
            p[:] = 0.0
    res = np.linalg.norm(b - matvec(x)) / bn
    return x, dict(iters=it, relres=res, converged=res <= tol)


def gmres(matvec, b, x0=None, tol=1e-12, restart=50, maxiter=100000):
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    bn = np.linalg.norm(b)
    if bn == 0.0:
        return np.zeros_like(b), dict(iters=0, relres=0.0, converged=True)
    it = 0
    while it < maxiter:
        r = b - matvec(x)
        beta = np.linalg.norm(r)
        if beta <= tol * bn:
            break
        k = restart
        V = np.zeros((k + 1, b.size))
        H = np.zeros((k + 1, k))
        cs = np.zeros(k)
        sn = np.zeros(k)
        g = np.zeros(k + 1)
        g[0] = beta
        V[0] = r / beta
        j_used = 0
        for j in range(k):
            w = matvec(V[j])
            for i in range(j + 1):            # modified Gram-Schmidt
                H[i, j] = np.dot(w, V[i])
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] > 0.0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):                # previous rotations
                tmp = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = tmp
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / den
            sn[j] = H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            j_used = j + 1
            it += 1
            if abs(g[j + 1]) <= tol * bn or it >= maxiter:
                break
        y = np.linalg.solve(np.triu(H[:j_used, :j_used]), g[:j_used])
        x = x + V[:j_used].T @ y
    res = np.linalg.norm(b - matvec(x)) / bn
    return x, dict(iters=it, relres=res, converged=res <= tol)


def gauge_matvec(matvec, n_s, gamma):
    """Rank-one gauge for a singular closed-surface Poisson system:
    (A + gamma 1 w^T) u with w = 1/n_s on the PDE DOFs and 0 on BC DOFs."""
    def mv(u):
        return matvec(u) + gamma * (np.sum(u[:n_s]) / n_s)
    return mv
