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


def implicit_surface(kind: str, params: dict):
    """Level-set function F (F = 0 on the surface) and its gradient, for the
    ellipsoid sum (x_i / a_i)^2 = 1 and the torus (sqrt(x^2 + y^2) - R)^2 + z^2 = r^2."""
    if kind in ("sphere", "ellipsoid"):
        ax = np.asarray(params.get("axes", (1.0, 1.0, 1.0)), dtype=np.float64)

        def F(x):
            return np.sum((x / ax) ** 2, axis=-1) - 1.0

        def G(x):
            return 2.0 * x / ax ** 2
        return F, G
    if kind == "torus":
        R, r = params["R"], params["r"]

        def F(x):
            rho = np.sqrt(x[..., 0] ** 2 + x[..., 1] ** 2)
            return (rho - R) ** 2 + x[..., 2] ** 2 - r * r

        def G(x):
            rho = np.sqrt(x[..., 0] ** 2 + x[..., 1] ** 2)
            k = 2.0 * (rho - R) / rho
            return np.stack([k * x[..., 0], k * x[..., 1], 2.0 * x[..., 2]], axis=-1)
        return F, G
    raise ValueError(kind)


def patch_integral(fun, F, G, a, b, c, p=None, n=24, h=1e-5):
    """Integral of fun(x) dA over the curved patch that a projection maps onto
    the flat triangle (a, b, c), from the definition of the area element.

    A point s of the triangle's plane (2-D coordinates in the frame e1 = b - a,
    e2 = n x e1) is carried to the surface along the line through it with
    direction n (p None: orthogonal projection) or s - p (central projection
    from p); the surface point x(s) is the root of F on that line nearest to
    s (Newton).  dA = |dx/ds1 x dx/ds2| ds1 ds2 with the derivatives taken by
    central differences of step h, and the plane integral is a Duffy
    Gauss-Legendre rule (`triangle_integral`).
    """
    nj = np.cross(b - a, c - a)
    nj = nj / np.linalg.norm(nj)
    e1 = (b - a) / np.linalg.norm(b - a)
    e2 = np.cross(nj, e1)

    def on_plane(s):
        return a + s[..., 0:1] * e1 + s[..., 1:2] * e2

    def X(s):
        xi = on_plane(s)
        d = np.broadcast_to(nj, xi.shape) if p is None else xi - p
        t = np.zeros(xi.shape[:-1])
        for _ in range(30):
            x = xi + t[..., None] * d
            t = t - F(x) / np.sum(G(x) * d, axis=-1)
        return xi + t[..., None] * d

    def integrand(s):
        d1 = np.array([h, 0.0])
        d2 = np.array([0.0, h])
        x1 = (X(s + d1) - X(s - d1)) / (2 * h)
        x2 = (X(s + d2) - X(s - d2)) / (2 * h)
        return fun(X(s)) * np.linalg.norm(np.cross(x1, x2), axis=-1)

    def to2(v):
        return np.array([np.dot(v - a, e1), np.dot(v - a, e2)])
    return triangle_integral(integrand, to2(a), to2(b), to2(c), n=n)
