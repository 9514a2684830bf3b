"""Independent closed forms and numerical rules used to pin the oracle.

Nothing here is imported by the oracle or the GPU library; each function is a
piece of mathematics that a test compares the oracle against.
"""
import math

import numpy as np


def rk4_amplification(z: float) -> float:
    """RK4 stability polynomial R(z) = 1 + z + z^2/2 + z^3/6 + z^4/24."""
    return 1.0 + z + z * z / 2.0 + z ** 3 / 6.0 + z ** 4 / 24.0


def sphere_kernel_integral(kind: int, p) -> float:
    """Integral over the unit sphere of a Mexican-hat w(|x - y|) dA(y).

    With rho = |x - y| one has dA = 2 pi rho drho, rho in [0, 2], so
      Gaussian  A exp(-rho^2/s^2):  pi A s^2 (1 - exp(-4/s^2))
      exponential A exp(-rho/s):    2 pi A s^2 (1 - exp(-2/s)(1 + 2/s)).
    """
    A_e, s_e, A_i, s_i = p
    if kind == 0:
        g = lambda A, s: math.pi * A * s * s * (1 - math.exp(-4 / (s * s)))
    else:
        g = lambda A, s: 2 * math.pi * A * s * s * (1 - math.exp(-2 / s) * (1 + 2 / s))
    return g(A_e, s_e) - g(A_i, s_i)


def sphere_monomial_integral(a: int, b: int, c: int) -> float:
    """Integral of x^a y^b z^c over the unit sphere (0 unless all exponents are even)."""
    if a % 2 or b % 2 or c % 2:
        return 0.0
    al, be, ga = (a + 1) / 2, (b + 1) / 2, (c + 1) / 2
    return 2 * math.gamma(al) * math.gamma(be) * math.gamma(ga) / math.gamma(al + be + ga)


def duffy_triangle_integral(fun, P, p, q, n=40):
    """Integral of fun over the 2-D triangle (P, p, q) by a Duffy map with apex P.

    s(u, v) = P + u (p - P) + u v (q - p),  ds = u |(p - P) x (q - P)| du dv,
    with Gauss-Legendre in u and v; a point singularity at P is smoothed away.
    """
    x, w = np.polynomial.legendre.leggauss(n)
    x = 0.5 * (x + 1)
    w = 0.5 * w
    U, V = np.meshgrid(x, x, indexing="ij")
    W = np.outer(w, w)
    pts = P + U[..., None] * (p - P) + (U * V)[..., None] * (q - p)
    jac = abs((p - P)[0] * (q - P)[1] - (p - P)[1] * (q - P)[0])
    return float(np.sum(W * U * jac * fun(pts)))


def triangle_integral(fun, v0, v1, v2, P=None, n=40):
    """Integral over triangle (v0, v1, v2), split at P (default: centroid) into three Duffy pieces."""
    if P is None:
        P = (v0 + v1 + v2) / 3
    def cross(a, b):
        return a[0] * b[1] - a[1] * b[0]
    o = np.sign(cross(v1 - v0, v2 - v0))
    tot = 0.0
    for a, b in ((v0, v1), (v1, v2), (v2, v0)):
        s = np.sign(cross(a - P, b - P)) * o
        if s != 0:
            tot += s * duffy_triangle_integral(fun, P, a, b, n)
    return tot


def ellipsoid_area_numeric(a, b, c, n=400):
    """Area of x^2/a^2 + y^2/b^2 + z^2/c^2 = 1 from |x_t x x_p| on a Gauss-Legendre x trapezoid grid."""
    t, wt = np.polynomial.legendre.leggauss(n)     # t = cos(polar)
    ph = 2 * np.pi * (np.arange(2 * n) + 0.5) / (2 * n)
    T, Pp = np.meshgrid(t, ph, indexing="ij")
    st = np.sqrt(1 - T * T)
    # x = (a st cos p, b st sin p, c t) with parameters (t, p): derivatives
    xt = np.stack([-a * T / st * np.cos(Pp), -b * T / st * np.sin(Pp), c * np.ones_like(T)], -1)
    xp = np.stack([-a * st * np.sin(Pp), b * st * np.cos(Pp), np.zeros_like(T)], -1)
    dA = np.linalg.norm(np.cross(xt, xp), axis=-1)
    return float(np.sum(dA * wt[:, None]) * (2 * np.pi / (2 * n)))
