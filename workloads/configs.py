"""The five synthetic workloads, generated from fixed seeds.

Each workload is a surface node set, Mexican-hat kernel parameters, a sigmoid
firing rate, initial states, a step size and a step count.  Workload k draws
every random number from ``numpy.random.default_rng(k)`` (PCG64), in the order
written in its builder, so the oracle and the GPU path see identical inputs.

Choices where the workload description leaves room (stated once here):

* a "Gaussian bump of width w and height h" centred at c is
  u(x) = h exp(-|x - c|^2 / w^2) in chordal distance, c a seeded node;
* "N(0, 0.01) noise" has standard deviation 0.01;
* the ellipsoid ensemble and the uneven batch use dt = 0.05 (their step size
  is not given; 0.05 is the step of the other Gaussian-kernel workload);
* uneven-batch parameter ranges: A_e ~ U(.8, 1.2), s_e ~ U(.12, .18),
  A_i ~ U(.4, .6), s_i ~ U(.3, .5), beta = 20, theta = 0.2.

Quadrature weights are *not* produced here: they belong to the method.  For
throughput runs, ``area_share_weights`` gives a stand-in rule (every node
weighted by |D|/N) whose values only serve as realistic-magnitude inputs.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import surfaces as S

GAUSS_MH = 0
EXP_MH = 1


@dataclass
class Workload:
    name: str
    surface: S.Surface
    kernel_kind: int
    kernel: tuple            # (A_e, s_e, A_i, s_i)
    beta: float
    theta: np.ndarray        # (B,) firing threshold per state
    u0: np.ndarray           # (B, N) float64: state b is row b (column-major N x B)
    dt: float
    steps: int
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.surface.n

    @property
    def b(self) -> int:
        return self.u0.shape[0]

    def pair_interactions(self) -> float:
        """N^2 * B per operator application, 4 applications per RK4 step."""
        return 4.0 * self.steps * float(self.n) ** 2 * self.b


def bump(xyz: np.ndarray, centre: np.ndarray, width: float = 0.3, height: float = 1.0) -> np.ndarray:
    d2 = np.sum((xyz - centre) ** 2, axis=1)
    return height * np.exp(-d2 / (width * width))


def surface_area(surface: S.Surface) -> float:
    """Area of the continuous surface (closed forms, or 2-D Gauss rules)."""
    kind, p = surface.kind, surface.params
    if kind == "sphere":
        return 4.0 * math.pi
    if kind == "torus":
        return 4.0 * math.pi ** 2 * p["R"] * p["r"]
    if kind == "ellipsoid":
        return ellipsoid_area(*p["axes"])
    if kind == "bumpy":
        return bumpy_area()
    raise ValueError(kind)


def ellipsoid_area(a: float, b: float, c: float) -> float:
    """Legendre's formula for a triaxial ellipsoid with a >= b >= c."""
    from scipy.special import ellipeinc, ellipkinc
    a, b, c = sorted((a, b, c), reverse=True)
    phi = math.acos(c / a)
    k2 = (a * a * (b * b - c * c)) / (b * b * (a * a - c * c))
    s = math.sin(phi)
    return 2 * math.pi * c * c + 2 * math.pi * a * b / s * (
        ellipeinc(phi, k2) * s * s + ellipkinc(phi, k2) * (c * c) / (a * a))


def bumpy_area(n_t: int = 200, n_p: int = 400) -> float:
    """Area of r = rho(u) by Gauss-Legendre in cos(polar) x trapezoid in azimuth.

    For x = rho(u) u:  dA = rho * sqrt(rho^2 + |grad_S rho|^2) dOmega.
    """
    t, wt = np.polynomial.legendre.leggauss(n_t)
    ph = 2 * np.pi * np.arange(n_p) / n_p
    T, P = np.meshgrid(t, ph, indexing="ij")
    st = np.sqrt(1 - T * T)
    u = np.stack([st * np.cos(P), st * np.sin(P), T], axis=-1).reshape(-1, 3)
    rho = S.bumpy_radius(u)
    k = S.BUMPY_EPS * S.Y42_C
    ux, uy, uz = u[:, 0], u[:, 1], u[:, 2]
    g = np.stack([k * (7 * uz * uz - 1) * 2 * ux, k * (7 * uz * uz - 1) * (-2 * uy),
                  k * 14 * uz * (ux * ux - uy * uy)], axis=1)
    g_t = g - np.sum(g * u, axis=1, keepdims=True) * u
    dA = rho * np.sqrt(rho * rho + np.sum(g_t * g_t, axis=1))
    return float(np.sum(dA.reshape(n_t, n_p) * wt[:, None]) * (2 * np.pi / n_p))


def area_share_weights(surface: S.Surface) -> np.ndarray:
    """Stand-in quadrature weights |D|/N (throughput inputs only)."""
    return np.full(surface.n, surface_area(surface) / surface.n)


# ----------------------------------------------------------------- workloads

def sphere_small(n: int = 2000) -> Workload:
    """Unit sphere, Fibonacci nodes, Gaussian Mexican hat, one state."""
    rng = np.random.default_rng(0)
    surf = S.sphere(n)
    c = surf.xyz[rng.integers(n)]
    u0 = bump(surf.xyz, c) + rng.normal(0.0, 0.01, size=n)
    return Workload("sphere-n%d-gauss-b1" % n, surf, GAUSS_MH, (1.0, 0.15, 0.5, 0.4),
                    20.0, np.array([0.2]), u0[None, :].copy(), 0.05, 50)


def torus_exp(n: int = 32768, steps: int = 500, seed: int = 1) -> Workload:
    """Torus R=1, r=0.4, jittered rings, exponential Mexican hat, two bumps."""
    rng = np.random.default_rng(seed)
    surf = S.torus(n, rng, 1.0, 0.4)
    idx = rng.integers(n, size=2)
    u0 = bump(surf.xyz, surf.xyz[idx[0]]) + bump(surf.xyz, surf.xyz[idx[1]])
    return Workload("torus-n%d-exp-b1" % n, surf, EXP_MH, (2.0, 0.1, 1.0, 0.3),
                    20.0, np.array([0.25]), u0[None, :].copy(), 0.02, steps)


def ellipsoid_ensemble(n: int = 65536, b: int = 64, steps: int = 200) -> Workload:
    """Ellipsoid (1, .8, .6), B states with one seeded bump and theta ~ U(.15, .3) each."""
    rng = np.random.default_rng(2)
    surf = S.ellipsoid(n, (1.0, 0.8, 0.6))
    centres = rng.integers(n, size=b)
    theta = rng.uniform(0.15, 0.3, size=b)
    u0 = np.stack([bump(surf.xyz, surf.xyz[c]) for c in centres])
    return Workload("ellipsoid-n%d-gauss-b%d" % (n, b), surf, GAUSS_MH, (1.0, 0.15, 0.5, 0.4),
                    20.0, theta, u0, 0.05, steps)


def uneven_batch(p: int = 48, n_lo: int = 1000, n_hi: int = 40000, steps: int = 100,
                 b_choices=(1, 4, 16)) -> list[Workload]:
    """P problems: N log-uniform, seeded surface kind, kernel parameters and B."""
    rng = np.random.default_rng(3)
    kinds = ("sphere", "torus", "ellipsoid", "bumpy")
    out = []
    for k in range(p):
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        kind = kinds[rng.integers(4)]
        b = int(b_choices[rng.integers(len(b_choices))])
        kern = (rng.uniform(0.8, 1.2), rng.uniform(0.12, 0.18),
                rng.uniform(0.4, 0.6), rng.uniform(0.3, 0.5))
        surf = S.make_surface(kind, n, rng)
        centres = rng.integers(n, size=b)
        u0 = np.stack([bump(surf.xyz, surf.xyz[c]) for c in centres])
        out.append(Workload("batch%02d-%s-n%d-b%d" % (k, kind, n, b), surf, GAUSS_MH,
                            tuple(float(v) for v in kern), 20.0, np.full(b, 0.2), u0,
                            0.05, steps))
    return out


def torus_adjoint(n: int = 16384, steps: int = 400, ckpt_every: int = 40) -> Workload:
    """Torus workload for gradients; the loss target uses perturbed parameters.

    Perturbation: p_target = p * (1 + 0.05 U(-1, 1)) for (A_e, s_e, A_i, s_i, theta).
    """
    w = torus_exp(n, steps, seed=4)
    rng = np.random.default_rng(40)
    base = np.array(list(w.kernel) + [w.theta[0]])
    pert = base * (1.0 + 0.05 * rng.uniform(-1.0, 1.0, size=5))
    dirs = rng.normal(size=(4, n))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    w.name = "torus-n%d-exp-adjoint" % n
    w.extra = {"target_params": pert, "ckpt_every": ckpt_every, "u0_dirs": dirs}
    return w


def bumpy_syndep(n: int = 20000, steps: int = 200) -> Workload:
    """Bumpy sphere with synaptic depression (the travelling-spot setting of the
    paper's section 5.2): the paper's normalised-Gaussian lateral inhibition
    A_e = 5, A_i = 7, sigma_e = .05, sigma_i = .1 rewritten as A exp(-r^2/s^2)
    (A = A_paper / (2 pi sigma^2), s = sqrt(2) sigma).  Not given in the paper,
    chosen here: sigmoid gain 20 and threshold 0.3, tau = 20, beta_d = 1,
    dt = 0.02, a(0) = 1, one bump of width 0.15 and height 1."""
    rng = np.random.default_rng(5)
    surf = S.bumpy_sphere(n)
    c = surf.xyz[rng.integers(n)]
    u0 = bump(surf.xyz, c, width=0.15)
    A_e, A_i, se, si = 5.0, 7.0, 0.05, 0.1
    kern = (A_e / (2 * math.pi * se * se), math.sqrt(2) * se, A_i / (2 * math.pi * si * si), math.sqrt(2) * si)
    return Workload("bumpy-syndep-n%d" % n, surf, GAUSS_MH, kern, 20.0, np.array([0.3]), u0[None, :].copy(), 0.02,
                    steps, extra={"tau": 20.0, "beta_d": 1.0, "a0": np.ones((1, n))})


def by_index(k: int, **kw):
    return [sphere_small, torus_exp, ellipsoid_ensemble, uneven_batch, torus_adjoint][k](**kw)
