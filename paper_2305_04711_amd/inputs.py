"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle
checks.  This module holds none of the closest point method's arithmetic: it
only evaluates smooth manifold data (real spherical harmonics on a sphere,
Fourier modes on a circle or torus) at given points, from seeded
coefficients.

Real spherical harmonics are orthonormal on the unit sphere, built from the
associated Legendre functions by the three-term recurrence in l.
"""

from math import factorial, pi, sqrt

import numpy as np


class _Torch:
    """The few numpy functions used below, for torch tensors (the same
    formulas evaluated on the GPU for large inputs)."""

    def __init__(self, torch):
        self.t = torch

    def asarray(self, a, dtype=None):
        return a if isinstance(a, self.t.Tensor) else self.t.tensor(a, dtype=self.t.float64)

    def sqrt(self, a):
        return self.t.sqrt(a)

    def arctan2(self, y, x):
        return self.t.atan2(y, x)

    def cos(self, a):
        return self.t.cos(a)

    def sin(self, a):
        return self.t.sin(a)

    def zeros_like(self, a):
        return self.t.zeros_like(a)

    def ones_like(self, a):
        return self.t.ones_like(a)

    def maximum0(self, a):
        return self.t.clamp(a, min=0.0)


def _xp(pts):
    if type(pts).__module__.startswith("torch"):
        import torch
        return _Torch(torch)
    return None


# ---------------------------------------------------------------- sphere
def _assoc_legendre(lmax, x, xp=None):
    """P[l][m](x) for 0 <= m <= l <= lmax, without the Condon-Shortley phase."""
    if xp is None:
        x = np.asarray(x, dtype=np.float64)
        s = np.sqrt(np.maximum(0.0, 1.0 - x * x))
        pmm = np.ones_like(x)
    else:
        s = xp.sqrt(xp.maximum0(1.0 - x * x))
        pmm = xp.ones_like(x)
    P = [[None] * (lmax + 1) for _ in range(lmax + 1)]
    for m in range(lmax + 1):
        if m > 0:
            pmm = pmm * (2 * m - 1) * s
        P[m][m] = pmm
        if m + 1 <= lmax:
            P[m + 1][m] = x * (2 * m + 1) * pmm
        for l in range(m + 2, lmax + 1):
            P[l][m] = ((2 * l - 1) * x * P[l - 1][m]
                       - (l + m - 1) * P[l - 2][m]) / (l - m)
    return P


def real_sph_harm(lmax, pts, center=(0.0, 0.0, 0.0)):
    """Dict (l, m) -> values of the orthonormal real spherical harmonic at the
    directions of pts - center.  m > 0 uses cos(m phi), m < 0 sin(|m| phi).
    pts may be a numpy array or a torch tensor."""
    xp = _xp(pts)
    M = np if xp is None else xp
    d0 = pts[:, 0] - center[0]
    d1 = pts[:, 1] - center[1]
    d2 = pts[:, 2] - center[2]
    rr = M.sqrt(d0 * d0 + d1 * d1 + d2 * d2)
    ct = d2 / rr
    phi = M.arctan2(d1, d0)
    P = _assoc_legendre(lmax, ct, xp)
    out = {}
    for l in range(lmax + 1):
        for m in range(0, l + 1):
            nrm = sqrt((2 * l + 1) / (4 * pi) * factorial(l - m) / factorial(l + m))
            if m == 0:
                out[(l, 0)] = nrm * P[l][0]
            else:
                out[(l, m)] = sqrt(2.0) * nrm * P[l][m] * M.cos(m * phi)
                out[(l, -m)] = sqrt(2.0) * nrm * P[l][m] * M.sin(m * phi)
    return out


def sphere_coeffs(seed, lmin=1, lmax=8):
    """c_lm ~ N(0, 1) for lmin <= l <= lmax, in (l, m) order m = -l..l."""
    rng = np.random.default_rng(seed)
    keys = [(l, m) for l in range(lmin, lmax + 1) for m in range(-l, l + 1)]
    return dict(zip(keys, rng.standard_normal(len(keys))))


def sphere_field(coeffs, pts, center=(0.0, 0.0, 0.0), scale=None):
    """sum c_lm Y_lm at pts; scale(l) multiplies each degree if given."""
    lmax = max(l for l, _ in coeffs)
    Y = real_sph_harm(lmax, pts, center)
    xp = _xp(pts)
    out = np.zeros(len(pts)) if xp is None else xp.zeros_like(pts[:, 0])
    for (l, m), c in coeffs.items():
        out += (c if scale is None else c * scale(l)) * Y[(l, m)]
    return out


# ---------------------------------------------------------------- circle
def circle_source(seed, pts, center=(0.0, 0.0)):
    """cos(3 theta) + 0.1 sum_{k=1..4} (a_k cos k theta + b_k sin k theta),
    a, b ~ N(0, 1) from the seed.  Returns (values, (a, b))."""
    rng = np.random.default_rng(seed)
    a = rng.standard_normal(4)
    b = rng.standard_normal(4)
    d = np.asarray(pts) - np.asarray(center)
    th = np.arctan2(d[:, 1], d[:, 0])
    f = np.cos(3 * th)
    for k in range(1, 5):
        f = f + 0.1 * (a[k - 1] * np.cos(k * th) + b[k - 1] * np.sin(k * th))
    return f, (a, b)


# ---------------------------------------------------------------- torus
def torus_angles(pts, R=1.0, center=(0.0, 0.0, 0.0)):
    """Toroidal angle phi (about the z axis) and poloidal angle theta."""
    xp = _xp(pts)
    M = np if xp is None else xp
    d0 = pts[:, 0] - center[0]
    d1 = pts[:, 1] - center[1]
    d2 = pts[:, 2] - center[2]
    phi = M.arctan2(d1, d0)
    qr = M.sqrt(d0 * d0 + d1 * d1)
    theta = M.arctan2(d2, qr - R)
    return phi, theta


def torus_coeffs(seed, kmax=4):
    """c_ab ~ N(0,1)/(1 + a^2 + b^2) for |a|, |b| <= kmax, cos and sin parts."""
    rng = np.random.default_rng(seed)
    out = {}
    for a in range(-kmax, kmax + 1):
        for b in range(-kmax, kmax + 1):
            w = 1.0 / (1.0 + a * a + b * b)
            out[(a, b)] = (w * rng.standard_normal(), w * rng.standard_normal())
    return out


def torus_field(coeffs, pts, R=1.0, center=(0.0, 0.0, 0.0)):
    xp = _xp(pts)
    M = np if xp is None else xp
    phi, theta = torus_angles(pts, R, center)
    out = np.zeros(len(pts)) if xp is None else xp.zeros_like(phi)
    for (a, b), (cc, cs) in coeffs.items():
        ang = a * phi + b * theta
        out = out + cc * M.cos(ang) + cs * M.sin(ang)
    return out


def meridian_dirichlet(pts, seed=2, R=1.0, center=(0.0, 0.0, 0.0)):
    """Smooth Dirichlet data on meridian circles: 0.5 + 0.25 cos(theta) plus a
    seeded perturbation of the poloidal modes 1..3."""
    _, theta = torus_angles(pts, R, center)
    rng = np.random.default_rng(seed)
    c = 0.05 * rng.standard_normal((3, 2))
    g = 0.5 + 0.25 * np.cos(theta)
    for k in range(1, 4):
        g = g + c[k - 1, 0] * np.cos(k * theta) + c[k - 1, 1] * np.sin(k * theta)
    return g


def random_vector(n, seed, dtype=np.float64):
    return np.random.default_rng(seed).standard_normal(n).astype(dtype)
