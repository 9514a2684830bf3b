"""Seeded synthetic surfaces and node sets.

This module only describes *inputs*: node coordinates on a closed surface,
the surface's exact unit normals, and (for the torus) the ring structure the
nodes were generated on.  It contains none of the neural-field method's
arithmetic (no quadrature weights, kernels, firing rates or time stepping), so
both the FP64 oracle and the GPU path may consume what it produces.

Surfaces (paper section 4, eq. torus, and the surfaces of the synthetic
workloads):

* unit sphere, spherical-Fibonacci nodes;
* ellipsoid with semi-axes (a, b, c): Fibonacci sphere points stretched by
  diag(a, b, c);
* "bumpy sphere" r = 1 + 0.1 Y(u), Y the real, orthonormal degree-4 order-2
  spherical harmonic (no Condon-Shortley phase), so r lies in [0.94, 1.06];
* torus with major radius R and minor radius r, parameterised as in the
  paper's eq. torus, with nodes on an area-weighted jittered ring grid.
"""
from __future__ import annotations

import math

import numpy as np

GOLDEN = (1.0 + math.sqrt(5.0)) / 2.0

# Real orthonormal Y_4^2 written in Cartesian form on the unit sphere:
#   Y(x, y, z) = C * (7 z^2 - 1) * (x^2 - y^2),
#   C = (15/2) * sqrt(2 * 9/(4 pi) * 2!/6!) = (15/2) / sqrt(80 pi).
Y42_C = 7.5 / math.sqrt(80.0 * math.pi)
BUMPY_EPS = 0.1


def fibonacci_sphere(n: int) -> np.ndarray:
    """Spherical-Fibonacci points: z_i = 1 - (2i+1)/n, phi_i = 2 pi i / golden."""
    if n < 1:
        raise ValueError("n must be >= 1")
    i = np.arange(n, dtype=np.float64)
    z = 1.0 - (2.0 * i + 1.0) / n
    phi = 2.0 * np.pi * i / GOLDEN
    s = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    return np.stack([s * np.cos(phi), s * np.sin(phi), z], axis=1)


def y42(u: np.ndarray) -> np.ndarray:
    """Real orthonormal Y_4^2 at unit vectors u (..., 3)."""
    x, y, z = u[..., 0], u[..., 1], u[..., 2]
    return Y42_C * (7.0 * z * z - 1.0) * (x * x - y * y)


def bumpy_radius(u: np.ndarray) -> np.ndarray:
    return 1.0 + BUMPY_EPS * y42(u)


class Surface:
    """A node set on a closed surface plus what is known exactly about it."""

    def __init__(self, kind: str, xyz: np.ndarray, normals: np.ndarray,
                 params: dict, star_shaped: bool, ring: np.ndarray | None = None,
                 angles: np.ndarray | None = None):
        self.kind = kind
        self.xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        self.normals = np.ascontiguousarray(normals, dtype=np.float64)
        self.params = dict(params)
        self.star_shaped = star_shaped
        self.ring = ring          # torus only: ring index of every node
        self.angles = angles      # torus only: (phi, theta) of every node

    @property
    def n(self) -> int:
        return self.xyz.shape[0]

    def normal_at(self, x: np.ndarray) -> np.ndarray:
        """Exact outward unit normal at points x (m, 3) lying on the surface."""
        return surface_normal(self.kind, self.params, x)


def surface_normal(kind: str, params: dict, x: np.ndarray) -> np.ndarray:
    x = np.asarray(x, dtype=np.float64)
    if kind == "sphere":
        nrm = x.copy()
    elif kind == "ellipsoid":
        a, b, c = params["axes"]
        nrm = x / np.array([a * a, b * b, c * c])
    elif kind == "torus":
        R = params["R"]
        phi = np.arctan2(x[:, 1], x[:, 0])
        centre = np.stack([R * np.cos(phi), R * np.sin(phi), np.zeros_like(phi)], axis=1)
        nrm = x - centre
    elif kind == "bumpy":
        # F(x) = |x| - rho(x/|x|);  grad F = u - (I - u u^T) grad rho(u) / |x|
        rad = np.linalg.norm(x, axis=1, keepdims=True)
        u = x / rad
        ux, uy, uz = u[:, 0], u[:, 1], u[:, 2]
        k = BUMPY_EPS * Y42_C
        g = np.stack([k * (7 * uz * uz - 1) * 2 * ux,
                      k * (7 * uz * uz - 1) * (-2 * uy),
                      k * 14 * uz * (ux * ux - uy * uy)], axis=1)
        g_t = g - np.sum(g * u, axis=1, keepdims=True) * u
        nrm = u - g_t / rad
    elif kind == "flat":
        nrm = np.zeros_like(x)
        nrm[:, 2] = 1.0
    else:
        raise ValueError(kind)
    return nrm / np.linalg.norm(nrm, axis=1, keepdims=True)


def sphere(n: int) -> Surface:
    x = fibonacci_sphere(n)
    return Surface("sphere", x, surface_normal("sphere", {}, x), {}, True)


def ellipsoid(n: int, axes=(1.0, 0.8, 0.6)) -> Surface:
    x = fibonacci_sphere(n) * np.asarray(axes, dtype=np.float64)
    p = {"axes": tuple(float(a) for a in axes)}
    return Surface("ellipsoid", x, surface_normal("ellipsoid", p, x), p, True)


def bumpy_sphere(n: int) -> Surface:
    u = fibonacci_sphere(n)
    x = u * bumpy_radius(u)[:, None]
    return Surface("bumpy", x, surface_normal("bumpy", {}, x), {}, True)


def _largest_remainder(shares: np.ndarray, total: int) -> np.ndarray:
    raw = shares / shares.sum() * total
    base = np.floor(raw).astype(np.int64)
    short = total - int(base.sum())
    order = np.argsort(-(raw - base), kind="stable")
    base[order[:short]] += 1
    return base


def torus(n: int, rng: np.random.Generator, R: float = 1.0, r: float = 0.4) -> Surface:
    """Area-weighted jittered ring grid on the torus of the paper's eq. torus.

    Rings sit at equal-area heights theta_k (R theta + r sin theta equispaced),
    ring k carries m_k ~ (R + r cos theta_k) nodes (largest-remainder rounding
    to n), nodes are equispaced in phi with a seeded ring offset, then jittered
    by U(-1/4, 1/4) of a cell in phi and in theta.  Draw order from `rng`:
    ring offsets, phi jitter, theta jitter.
    """
    if not (R > r > 0):
        raise ValueError("need R > r > 0")
    n_rings = max(3, int(round(math.sqrt(n * r / R))))
    if n < 3 * n_rings:
        raise ValueError("n too small for a ring grid")
    # equal-area ring heights: F(theta) = R theta + r sin theta on [-pi, pi)
    targets = -math.pi * R + (np.arange(n_rings) + 0.5) * (2.0 * math.pi * R / n_rings)
    th = targets / R
    for _ in range(60):
        th = th - (R * th + r * np.sin(th) - targets) / (R + r * np.cos(th))
    m = _largest_remainder(R + r * np.cos(th), n)
    if np.any(m < 3):
        raise ValueError("ring with fewer than 3 nodes")
    offsets = rng.uniform(0.0, 1.0, size=n_rings)
    ring = np.repeat(np.arange(n_rings), m)
    slot = np.concatenate([np.arange(mk) for mk in m]).astype(np.float64)
    mk = m[ring].astype(np.float64)
    jphi = rng.uniform(-0.25, 0.25, size=n)
    jth = rng.uniform(-0.25, 0.25, size=n)
    phi = 2.0 * np.pi * (slot + offsets[ring] + jphi) / mk
    dth = (2.0 * math.pi * R / n_rings) / (R + r * np.cos(th))   # local ring spacing
    theta = th[ring] + jth * dth[ring]
    phi = np.mod(phi, 2.0 * np.pi)
    x = np.stack([(R + r * np.cos(theta)) * np.cos(phi),
                  (R + r * np.cos(theta)) * np.sin(phi),
                  r * np.sin(theta)], axis=1)
    p = {"R": float(R), "r": float(r)}
    return Surface("torus", x, surface_normal("torus", p, x), p, False,
                   ring=ring, angles=np.stack([phi, theta], axis=1))


def flat_square(n: int, L: float = 2.0 * math.pi, rng: np.random.Generator | None = None,
                jitter: float = 0.0) -> Surface:
    """Nodes on the square [-L/2, L/2]^2 in the plane z = 0 (the flat domains of
    the paper's section 4): equispaced boundary nodes (corners included) and
    interior nodes on a near-equilateral triangular lattice, rows offset by half
    a spacing.  With rng and jitter > 0 every interior node moves by
    U(-jitter, jitter) of a spacing in x and in y (drawn in that order).
    The node count is close to n, not equal to it.
    """
    c = 2.0 / math.sqrt(3.0)
    m = (-4.0 + math.sqrt(16.0 + 4.0 * c * n)) / (2.0 * c)      # L / h for ~n nodes
    nb = max(2, int(round(m)))                                 # boundary segments per side
    nr = max(1, int(round(m * c)))                             # interior rows
    nc = max(1, int(round(m)))                                 # interior columns
    hx, hy = L / nc, L / nr
    k = np.repeat(np.arange(nr), nc)
    j = np.tile(np.arange(nc), nr)
    xi = -L / 2 + (j + 0.25 + 0.5 * (k % 2)) * hx
    yi = -L / 2 + (k + 0.5) * hy
    if rng is not None and jitter > 0:
        xi = xi + rng.uniform(-jitter, jitter, size=xi.size) * hx
        yi = yi + rng.uniform(-jitter, jitter, size=yi.size) * hy
    t = -L / 2 + L * np.arange(nb) / nb
    edge = np.concatenate([np.stack([t, np.full(nb, -L / 2)], 1),          # bottom, left to right
                           np.stack([np.full(nb, L / 2), t], 1),           # right, bottom to top
                           np.stack([-t, np.full(nb, L / 2)], 1),          # top, right to left
                           np.stack([np.full(nb, -L / 2), -t], 1)])        # left, top to bottom
    xy = np.concatenate([edge, np.stack([xi, yi], 1)])
    x = np.concatenate([xy, np.zeros((xy.shape[0], 1))], axis=1)
    p = {"L": float(L), "n_boundary": int(edge.shape[0])}
    return Surface("flat", x, surface_normal("flat", p, x), p, False)


def make_surface(kind: str, n: int, rng: np.random.Generator, **kw) -> Surface:
    if kind == "sphere":
        return sphere(n)
    if kind == "ellipsoid":
        return ellipsoid(n, **kw)
    if kind == "bumpy":
        return bumpy_sphere(n)
    if kind == "torus":
        return torus(n, rng, **kw)
    raise ValueError(kind)
