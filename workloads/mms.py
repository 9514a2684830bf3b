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
