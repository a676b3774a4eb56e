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


# ---------------------------------------------------------------- sphere
def _assoc_legendre(lmax, x):
    """P[l][m](x) for 0 <= m <= l <= lmax, without the Condon-Shortley phase."""
    x = np.asarray(x, dtype=np.float64)
    s = np.sqrt(np.maximum(0.0, 1.0 - x * x))
    P = [[None] * (lmax + 1) for _ in range(lmax + 1)]
    pmm = np.ones_like(x)
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
    directions of pts - center.  m > 0 uses cos(m phi), m < 0 sin(|m| phi)."""
    d = np.asarray(pts, dtype=np.float64) - np.asarray(center)
    rr = np.sqrt(np.sum(d * d, axis=1))
    ct = d[:, 2] / rr
    phi = np.arctan2(d[:, 1], d[:, 0])
    P = _assoc_legendre(lmax, ct)
    out = {}
    for l in range(lmax + 1):
        for m in range(0, l + 1):
            nrm = sqrt((2 * l + 1) / (4 * pi) * factorial(l - m) / factorial(l + m))
            if m == 0:
                out[(l, 0)] = nrm * P[l][0]
            else:
                out[(l, m)] = sqrt(2.0) * nrm * P[l][m] * np.cos(m * phi)
                out[(l, -m)] = sqrt(2.0) * nrm * P[l][m] * np.sin(m * phi)
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
    out = np.zeros(len(pts))
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
    d = np.asarray(pts, dtype=np.float64) - np.asarray(center)
    phi = np.arctan2(d[:, 1], d[:, 0])
    qr = np.sqrt(d[:, 0] ** 2 + d[:, 1] ** 2)
    theta = np.arctan2(d[:, 2], qr - R)
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
    phi, theta = torus_angles(pts, R, center)
    out = np.zeros(len(pts))
    for (a, b), (cc, cs) in coeffs.items():
        ang = a * phi + b * theta
        out += cc * np.cos(ang) + cs * np.sin(ang)
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
