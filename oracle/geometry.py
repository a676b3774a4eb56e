"""Analytic closest-point functions (Sec. 3.1 definition of cp_S as the
arg-min of Euclidean distance; App. A: analytic expressions are used where they
exist).

Each function takes points as an (n, d) FP64 array and returns an (n, d) FP64
array.  The formulas are evaluated in the order written, with only +, -, *, /
and sqrt (all correctly rounded in IEEE FP64), so the result does not depend on
the machine.  Points where the closest point is not unique (the centre of a
circle or sphere, the axis of a torus) give NaN, which fails every distance
test and so never enters a band.

An interior boundary C also carries a fixed orientation vector o_C, used only
for the on-C tie rule of Sec. 4.2 (a closest point within 0.1 h^2 of C "can be
assigned to either side"; the oracle assigns it to the side o_C points to).
"""

import numpy as np

_ERR = dict(divide="ignore", invalid="ignore")


class Circle:
    """Circle of radius R about (cx, cy) in R^2."""

    dim = 2

    def __init__(self, R=1.0, center=(0.0, 0.0)):
        self.R = float(R)
        self.c = np.asarray(center, dtype=np.float64)
        self.extent = np.array([self.R, self.R])
        self.reach = self.R

    def cp(self, X):
        with np.errstate(**_ERR):
            dx = X[:, 0] - self.c[0]
            dy = X[:, 1] - self.c[1]
            rho = np.sqrt(dx * dx + dy * dy)
            s = self.R / rho
            return np.stack([self.c[0] + dx * s, self.c[1] + dy * s], axis=1)


class Sphere:
    """Sphere of radius R about c in R^3."""

    dim = 3

    def __init__(self, R=1.0, center=(0.0, 0.0, 0.0)):
        self.R = float(R)
        self.c = np.asarray(center, dtype=np.float64)
        self.extent = np.array([self.R, self.R, self.R])
        self.reach = self.R

    def cp(self, X):
        with np.errstate(**_ERR):
            dx = X[:, 0] - self.c[0]
            dy = X[:, 1] - self.c[1]
            dz = X[:, 2] - self.c[2]
            rho = np.sqrt((dx * dx + dy * dy) + dz * dz)
            s = self.R / rho
            return np.stack([self.c[0] + dx * s, self.c[1] + dy * s,
                             self.c[2] + dz * s], axis=1)


class Torus:
    """Torus about the z axis through c: tube radius rho around the circle of
    radius R in the plane z = c_z.  The closest point is found in two steps:
    the nearest point q of the core circle, then the point at distance rho from
    q towards x."""

    dim = 3

    def __init__(self, R=1.0, rho=0.4, center=(0.0, 0.0, 0.0)):
        self.R = float(R)
        self.rho = float(rho)
        self.c = np.asarray(center, dtype=np.float64)
        self.extent = np.array([self.R + self.rho, self.R + self.rho, self.rho])
        self.reach = min(self.rho, self.R - self.rho)

    def cp(self, X):
        with np.errstate(**_ERR):
            dx = X[:, 0] - self.c[0]
            dy = X[:, 1] - self.c[1]
            dz = X[:, 2] - self.c[2]
            qr = np.sqrt(dx * dx + dy * dy)
            s = self.R / qr
            qx = dx * s
            qy = dy * s
            ex = dx - qx
            ey = dy - qy
            e = np.sqrt((ex * ex + ey * ey) + dz * dz)
            t = self.rho / e
            return np.stack([self.c[0] + (qx + ex * t),
                             self.c[1] + (qy + ey * t),
                             self.c[2] + dz * t], axis=1)


# ---------------------------------------------------------------------------
# Interior boundaries C (Sec. 4): closest point cp_C and orientation o_C.
# ---------------------------------------------------------------------------

class PointC:
    """A point C = p on S (Sec. 4, Fig. 3; Sec. 4.5 for R^3).  cp_C is the
    constant p.  o_C is supplied by the caller (for a point on a circle: the
    counter-clockwise tangent)."""

    def __init__(self, p, orient):
        self.p = np.asarray(p, dtype=np.float64)
        self.o = np.asarray(orient, dtype=np.float64)

    def cp(self, X):
        return np.broadcast_to(self.p, X.shape).copy()

    def orient(self, CPC):
        return np.broadcast_to(self.o, CPC.shape).copy()


class LatitudeC:
    """The circle where the sphere (centre c, radius R) meets the plane
    z = c_z + z0.  cp_C scales the horizontal offset of x to radius
    rho0 = sqrt(R^2 - z0^2).  o_C is the unit tangent of the sphere at cp_C
    pointing north (increasing z), which is normal to S_perp along C."""

    def __init__(self, sphere, z0):
        self.c = sphere.c
        self.R = sphere.R
        self.z0 = float(z0)
        self.rho0 = np.sqrt(self.R * self.R - self.z0 * self.z0)

    def cp(self, X):
        with np.errstate(**_ERR):
            dx = X[:, 0] - self.c[0]
            dy = X[:, 1] - self.c[1]
            q = np.sqrt(dx * dx + dy * dy)
            s = self.rho0 / q
            return np.stack([self.c[0] + dx * s, self.c[1] + dy * s,
                             np.full(X.shape[0], self.c[2] + self.z0)], axis=1)

    def orient(self, CPC):
        # horizontal unit direction u of cp_C, then (-z0 u, rho0) / R.
        ux = (CPC[:, 0] - self.c[0]) / self.rho0
        uy = (CPC[:, 1] - self.c[1]) / self.rho0
        return np.stack([(-self.z0 * ux) / self.R, (-self.z0 * uy) / self.R,
                         np.full(CPC.shape[0], self.rho0 / self.R)], axis=1)


class LatitudeArc(LatitudeC):
    """An open arc of the latitude circle (Sec. 4.4, open curves C): the
    points of the circle whose horizontal direction lies counter-clockwise
    from the unit direction a to the unit direction b.  cp_C is the circle's
    closest point when x's horizontal direction lies in the arc and the
    nearer endpoint otherwise (squared distances compared, ties to the start).
    at_boundary(X) flags Omega(dC), the nodes whose cp_C is an endpoint
    (eq. IBC_boundary_set)."""

    def __init__(self, sphere, z0, a, b):
        super().__init__(sphere, z0)
        self.a = np.asarray(a, dtype=np.float64)
        self.b = np.asarray(b, dtype=np.float64)

    def _inside(self, X):
        dx = X[:, 0] - self.c[0]
        dy = X[:, 1] - self.c[1]
        a0, a1 = self.a
        b0, b1 = self.b
        ca = a0 * dy - a1 * dx          # a x u
        cb = dx * b1 - dy * b0          # u x b
        if a0 * b1 - a1 * b0 >= 0.0:     # arc of at most a half turn
            return (ca >= 0.0) & (cb >= 0.0)
        return (ca >= 0.0) | (cb >= 0.0)

    def endpoints(self):
        z = self.c[2] + self.z0
        e0 = np.array([self.c[0] + self.rho0 * self.a[0], self.c[1] + self.rho0 * self.a[1], z])
        e1 = np.array([self.c[0] + self.rho0 * self.b[0], self.c[1] + self.rho0 * self.b[1], z])
        return e0, e1

    def cp(self, X):
        P = super().cp(X)
        inside = self._inside(X)
        e0, e1 = self.endpoints()
        D0, D1 = X - e0, X - e1
        d0 = (D0[:, 0] * D0[:, 0] + D0[:, 1] * D0[:, 1]) + D0[:, 2] * D0[:, 2]
        d1 = (D1[:, 0] * D1[:, 0] + D1[:, 1] * D1[:, 1]) + D1[:, 2] * D1[:, 2]
        E = np.where((d1 < d0)[:, None], e1, e0)
        return np.where(inside[:, None], P, E)

    def at_boundary(self, X):
        return ~self._inside(X)


class MeridianC:
    """A meridian (poloidal) circle of a torus: the tube circle in the vertical
    plane through the torus axis with horizontal unit direction (ex, ey).  Its
    centre is c0 = c + R (ex, ey, 0).  cp_C projects x - c0 onto that plane and
    scales the result to length rho.  o_C = e_z x (ex, ey, 0) = (-ey, ex, 0) is
    the normal of the plane, which contains S_perp along C."""

    def __init__(self, torus, ex, ey):
        self.c = torus.c
        self.R = torus.R
        self.rho = torus.rho
        self.ex = float(ex)
        self.ey = float(ey)

    def cp(self, X):
        with np.errstate(**_ERR):
            c0x = self.c[0] + self.R * self.ex
            c0y = self.c[1] + self.R * self.ey
            dx = X[:, 0] - c0x
            dy = X[:, 1] - c0y
            dz = X[:, 2] - self.c[2]
            a = dx * self.ex + dy * self.ey
            nrm = np.sqrt(a * a + dz * dz)
            s = self.rho / nrm
            a_s = a * s
            return np.stack([c0x + a_s * self.ex, c0y + a_s * self.ey,
                             self.c[2] + dz * s], axis=1)

    def orient(self, CPC):
        return np.broadcast_to(np.array([-self.ey, self.ex, 0.0]), CPC.shape).copy()


def band_radius_factor(dim, p=3, q=1):
    """Squared tube radius in units of h^2, eq. (bandwidth):
    (d-1)((p+1)/2)^2 + (q+(p+1)/2)^2.  For p = 3, q = 1: 13 in R^2, 17 in R^3."""
    a = (p + 1) / 2.0
    return (dim - 1) * a * a + (q + a) * (q + a)
