"""Closed-form manifold solutions used to pin the oracle (and, through it, the
GPU path).  Each is written from the mathematics, not from the CPM code.

* ``circle_point_dirichlet``: -u'' = f on the unit circle with u = 0 at the
  point theta = 0, for f a trigonometric polynomial; solved term by term on
  (0, 2 pi) with u(0) = u(2 pi) = 0:
  cos k th -> (cos k th - 1)/k^2, sin k th -> sin k th / k^2,
  a0 -> a0 th (2 pi - th) / 2.
* ``jump_exact``: the two-sided jump problem of Sec. 6.1.
* ``sphere_poisson``: -Delta_S u = sum f_lm Y_lm  =>  u = sum f_lm Y_lm/(l(l+1))
  up to a constant; ``sphere_screened`` divides by l(l+1) + 1.
* ``latitude_harmonic``: harmonic on the unit sphere minus the circle z = z0
  with u = sin(2 phi) on the circle.  Harmonic functions are invariant under
  the conformal stereographic map, and r^(+-2) sin(2 phi) are harmonic in the
  plane, so with q = (1 - z)/(1 + z): u = (q/q0) sin 2phi for z >= z0 and
  (q0/q) sin 2phi for z <= z0.
* ``torus_manufactured``: u = cos(phi) sin(theta) + 0.5 cos(2 theta) on the
  torus (R, rho) with Laplace-Beltrami, W = R + rho cos(theta):
  Delta u = u_phiphi / W^2 + u_thth / rho^2 - sin(theta) u_th / (rho W).
"""

import numpy as np

from paper_2305_04711_amd import inputs


def circle_point_dirichlet(theta, a0, ca, sa):
    """u for f = a0 + sum_k ca[k-1] cos k th + sa[k-1] sin k th, u(0) = 0."""
    th = np.mod(theta, 2 * np.pi)
    u = a0 * th * (2 * np.pi - th) / 2.0
    for k in range(1, len(ca) + 1):
        u = u + ca[k - 1] * (np.cos(k * th) - 1.0) / k ** 2
        u = u + sa[k - 1] * np.sin(k * th) / k ** 2
    return u


def jump_exact(theta, theta_c):
    s = np.mod(theta - theta_c, 2 * np.pi)
    return 2.0 * np.cos(theta - theta_c) + (10.0 / np.pi) * s


def sphere_poisson(coeffs, pts):
    return inputs.sphere_field(coeffs, pts, scale=lambda l: 1.0 / (l * (l + 1)))


def sphere_screened(coeffs, pts):
    return inputs.sphere_field(coeffs, pts, scale=lambda l: 1.0 / (l * (l + 1) + 1))


def latitude_harmonic(pts, z0):
    z = pts[:, 2]
    phi = np.arctan2(pts[:, 1], pts[:, 0])
    with np.errstate(divide="ignore", invalid="ignore"):
        q = (1 - z) / (1 + z)
        q0 = (1 - z0) / (1 + z0)
        amp = np.where(z >= z0, q / q0, q0 / q)
    return amp * np.sin(2 * phi)


def torus_manufactured(pts, R, rho):
    """(u, -Delta_S u) for the manufactured torus field."""
    phi, th = inputs.torus_angles(pts, R)
    W = R + rho * np.cos(th)
    u = np.cos(phi) * np.sin(th) + 0.5 * np.cos(2 * th)
    u_pp = -np.cos(phi) * np.sin(th)
    u_t = np.cos(phi) * np.cos(th) - np.sin(2 * th)
    u_tt = -np.cos(phi) * np.sin(th) - 2.0 * np.cos(2 * th)
    lap = u_pp / W ** 2 + u_tt / rho ** 2 - np.sin(th) * u_t / (rho * W)
    return u, -lap


def fit_slope(hs, errs):
    return np.polyfit(np.log(hs), np.log(errs), 1)[0]


def equator_split(pts, side):
    """Screened Poisson -Delta u + u = f on the unit sphere with a zero-Neumann
    interior boundary on the equator: u = x on the north side (side +1) and
    u = x + 3 z^2 + 6 on the south side.  Both satisfy the Neumann condition
    (the z-derivative of 3 z^2 vanishes at z = 0; x is even in z), x is an
    l = 1 harmonic (-Delta x = 2 x) and 3 z^2 + 6 = (3 z^2 - 1) + 7 combines
    an l = 2 harmonic (eigenvalue 6) with a constant, so
    f = 3 x on the north side and 3 x + 7 (3 z^2 - 1) + 7 = 3 x + 21 z^2 on
    the south side: f is continuous across the equator while u jumps by 6.
    Returns (u, f)."""
    pts = np.asarray(pts, dtype=np.float64)
    x, z = pts[:, 0], pts[:, 2]
    south = np.asarray(side) < 0
    u = x + np.where(south, 3.0 * z * z + 6.0, 0.0)
    f = 3.0 * x + np.where(south, 21.0 * z * z, 0.0)
    return u, f


def heat_l1(pts, t, axis=2):
    """u(x, t) = exp(-2 t) x_axis on the unit sphere: the l = 1 solution of
    u_t = Delta_S u (the paper's heat test with axis = 2, the polar cosine)."""
    return np.exp(-2.0 * t) * np.asarray(pts, dtype=np.float64)[:, axis]
