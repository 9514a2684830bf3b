"""A manufactured solution on the unit sphere (the method of manufactured
solutions of the paper's section 4, eq. manufactured_system, moved from the
flat square to the sphere).

The firing-rate field is chosen affine in y.e:
    phi(t, y) = f(u(t, y)) = a(t) + b(t) (y . e),
so that, by the Funk-Hecke theorem, for any radial kernel
    int_S2 w(|x - y|) phi(t, y) dA(y) = kappa0 a(t) + kappa1 b(t) (x . e),
    kappa_l = 2 pi int_{-1}^{1} w(sqrt(2 - 2 s)) P_l(s) ds   (P_0 = 1, P_1 = s).
With u = f^{-1}(phi) for the sigmoid f(u) = 1 / (1 + exp(-beta (u - theta))),
the forcing
    F(t, x) = d_t u + u - kappa0 a(t) - kappa1 b(t) (x . e)
makes u an exact solution of u_t = -u + int w f(u) dA + F.  This module only
builds inputs (exact states and forcing arrays); it contains none of the
discrete method.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.integrate import quad

from . import surfaces as S


def kernel_radial(kind: int, p, r):
    A_e, s_e, A_i, s_i = p
    if kind == 0:
        return A_e * math.exp(-(r / s_e) ** 2) - A_i * math.exp(-(r / s_i) ** 2)
    return A_e * math.exp(-r / s_e) - A_i * math.exp(-r / s_i)


def funk_hecke(kind: int, p, degree: int) -> float:
    leg = (lambda s: 1.0) if degree == 0 else (lambda s: s)
    val, _ = quad(lambda s: kernel_radial(kind, p, math.sqrt(max(0.0, 2.0 - 2.0 * s))) * leg(s), -1.0, 1.0,
                  epsabs=1e-14, epsrel=1e-13, limit=400, points=[1.0 - 1e-3, 1.0 - 1e-2, 1.0 - 1e-1])
    return 2.0 * math.pi * val


class SphereMMS:
    """u(t, x) = f^{-1}(a(t) + b(t) x.e), a = a0 + a1 sin(w t), b = b1 cos(w t)."""

    def __init__(self, n: int, kind: int = 0, kernel=(1.0, 0.15, 0.5, 0.4), beta: float = 5.0,
                 theta: float = 0.5, omega: float = 2.0, a0=0.5, a1=0.1, b1=0.3,
                 e=(0.3, -0.5, 0.812403840463596)):
        self.surface = S.sphere(n)
        self.kind, self.kernel = kind, tuple(kernel)
        self.beta, self.theta, self.omega = beta, theta, omega
        self.a0, self.a1, self.b1 = a0, a1, b1
        e = np.asarray(e, dtype=np.float64)
        self.e = e / np.linalg.norm(e)
        self.kappa0 = funk_hecke(kind, kernel, 0)
        self.kappa1 = funk_hecke(kind, kernel, 1)
        self.xe = self.surface.xyz @ self.e

    def ab(self, t):
        w = self.omega
        return (self.a0 + self.a1 * math.sin(w * t), self.b1 * math.cos(w * t),
                self.a1 * w * math.cos(w * t), -self.b1 * w * math.sin(w * t))

    def u(self, t):
        a, b, _, _ = self.ab(t)
        phi = a + b * self.xe
        return self.theta + np.log(phi / (1.0 - phi)) / self.beta

    def forcing(self, t):
        a, b, da, db = self.ab(t)
        phi = a + b * self.xe
        ut = (da + db * self.xe) / (self.beta * phi * (1.0 - phi))
        return ut + self.u(t) - self.kappa0 * a - self.kappa1 * b * self.xe

    def stage_forcing(self, dt: float, steps: int) -> np.ndarray:
        """(steps, 3, 1, N): F at t_n, t_n + dt/2, t_n + dt for each RK4 step."""
        out = np.empty((steps, 3, 1, self.surface.n))
        for k in range(steps):
            t = k * dt
            out[k, 0, 0] = self.forcing(t)
            out[k, 1, 0] = self.forcing(t + 0.5 * dt)
            out[k, 2, 0] = self.forcing(t + dt)
        return out


class FlatMMS:
    """A manufactured solution on the doubly periodic square [-L/2, L/2]^2 (the
    flat setting of the paper's section 4, eq. manufactured_system, with the
    periodic distance of eq. dist and the normalised Gaussian of eq. gauss).

    The firing-rate field is a trigonometric polynomial whose centre circles
    like the paper's x_0(t) = (cos t / 5, sin t / 5):
        phi(t, x) = c0 + c1 (1 + cos(x - X(t))) (1 + cos(y - Y(t))),
    with L = 2 pi.  For the Gaussian Gauss(x, y; sigma) of total mass one, each
    Fourier mode exp(i k.y) is mapped to exp(-sigma^2 |k|^2 / 2) exp(i k.x)
    (the part of the Gaussian beyond the half period, exp(-pi^2 / (2 sigma^2)),
    is below FP64 resolution for sigma <= 1/4), so
        int w phi dy = c0 + c1 (1 + g1 (cos a + cos b) + g2 cos a cos b),
        a = x - X, b = y - Y, g1 = exp(-sigma^2 / 2), g2 = exp(-sigma^2).
    The paper's firing rate has gain 5 and threshold 1/2.  The kernel in the
    library's form: A_e = 1 / (2 pi sigma^2), s_e = sqrt(2) sigma, A_i = 0.
    """

    L = 2.0 * math.pi

    def __init__(self, n: int, sigma: float = 0.25, beta: float = 5.0, theta: float = 0.5,
                 c0: float = 0.1, c1: float = 0.2, rng: np.random.Generator | None = None, jitter: float = 0.0):
        if sigma > 0.25:
            raise ValueError("sigma above 1/4: the periodic wrap of the Gaussian is no longer negligible")
        self.surface = S.flat_square(n, self.L, rng, jitter)
        self.sigma, self.beta, self.theta, self.c0, self.c1 = sigma, beta, theta, c0, c1
        self.kind = 0
        self.kernel = (1.0 / (2.0 * math.pi * sigma * sigma), math.sqrt(2.0) * sigma, 0.0, 1.0)
        self.g1 = math.exp(-sigma * sigma / 2.0)
        self.g2 = math.exp(-sigma * sigma)
        self.x = self.surface.xyz[:, 0]
        self.y = self.surface.xyz[:, 1]

    @staticmethod
    def centre(t):
        return math.cos(t) / 5.0, math.sin(t) / 5.0, -math.sin(t) / 5.0, math.cos(t) / 5.0

    def phi(self, t):
        X, Y, _, _ = self.centre(t)
        return self.c0 + self.c1 * (1.0 + np.cos(self.x - X)) * (1.0 + np.cos(self.y - Y))

    def u(self, t):
        ph = self.phi(t)
        return self.theta + np.log(ph / (1.0 - ph)) / self.beta

    def K_phi(self, t):
        """The exact nonlocal term int_D w(dist(x, y)) phi(t, y) dy at the nodes."""
        X, Y, _, _ = self.centre(t)
        ca, cb = np.cos(self.x - X), np.cos(self.y - Y)
        return self.c0 + self.c1 * (1.0 + self.g1 * (ca + cb) + self.g2 * ca * cb)

    def forcing(self, t):
        X, Y, dX, dY = self.centre(t)
        a, b = self.x - X, self.y - Y
        ph = self.phi(t)
        dph = self.c1 * (np.sin(a) * dX * (1.0 + np.cos(b)) + (1.0 + np.cos(a)) * np.sin(b) * dY)
        ut = dph / (self.beta * ph * (1.0 - ph))
        return ut + self.u(t) - self.K_phi(t)

    def stage_forcing(self, dt: float, steps: int) -> np.ndarray:
        """(steps, 3, 1, N): F at t_n, t_n + dt/2, t_n + dt for each RK4 step."""
        out = np.empty((steps, 3, 1, self.surface.n))
        for k in range(steps):
            t = k * dt
            out[k, 0, 0] = self.forcing(t)
            out[k, 1, 0] = self.forcing(t + 0.5 * dt)
            out[k, 2, 0] = self.forcing(t + dt)
        return out
