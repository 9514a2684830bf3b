"""Pins for the oracle's flat periodic setting (CPU only).

* the doubly periodic distance (eq. dist) against a brute-force minimum over 25
  lattice shifts, written as plain loops, and against hand-worked cases;
* the planar RBF-QF rule on the square: exact for every polynomial of degree
  <= 2 (the rule's reproduction property), and convergent for a smooth
  non-polynomial integrand whose integral has a closed form;
* the flat manufactured solution: its nonlocal term against a periodic
  trapezoid sum on a fine uniform grid (spectrally accurate for this periodic
  integrand, and independent of RBF-QF), its time derivative against a
  central difference, and the forced discrete system converging to it;
* the discrete adjoint with the periodic distance against finite differences.
"""
import math

import numpy as np

from oracle import neural_field as NF
from oracle import quadrature as Q
from workloads import mms
from workloads import surfaces as S

L = 2.0 * math.pi


def test_periodic_distance_matches_bruteforce_over_25_shifts():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.uniform(-L / 2, L / 2, size=(25, 2)), rng.normal(0, 0.1, size=(25, 1))], axis=1)
    x[0] = (-L / 2, -L / 2, 0.0)
    x[1] = (L / 2, L / 2, 0.0)
    got = NF.distances(x, np.arange(25), L)
    for a in range(25):
        for b in range(25):
            best = math.inf
            for i in range(-2, 3):
                for j in range(-2, 3):
                    d = (x[a, 0] - x[b, 0] + i * L, x[a, 1] - x[b, 1] + j * L, x[a, 2] - x[b, 2])
                    best = min(best, math.sqrt(d[0] ** 2 + d[1] ** 2 + d[2] ** 2))
            assert abs(got[a, b] - best) <= 1e-14 * L
    assert got[0, 1] <= 1e-14 * L                     # opposite corners are one point of the torus
    assert np.allclose(got, got.T, rtol=0, atol=1e-15)


def test_periodic_distance_hand_cases_and_lattice_invariance():
    eps = 0.01
    x = np.array([[-L / 2 + eps, 0.3, 0.0], [L / 2 - eps, 0.3, 0.0], [0.0, 0.0, 0.0], [1.0, -L / 2 + 0.5, 0.0]])
    d = NF.distances(x, np.arange(4), L)
    assert abs(d[0, 1] - 2 * eps) < 1e-14
    assert abs(d[2, 3] - math.hypot(1.0, L / 2 - 0.5)) < 1e-14
    plain = NF.distances(x, np.arange(4))
    assert abs(plain[0, 1] - (L - 2 * eps)) < 1e-14
    shifted = x.copy()
    shifted[3, 0] -= L                                # the same point of the torus
    d2 = NF.distances(shifted, np.arange(4), L)
    assert np.allclose(d2, d, rtol=0, atol=1e-13)


def _square_monomial_integral(a, b):
    def one(k):
        return 0.0 if k % 2 else 2.0 * (L / 2) ** (k + 1) / (k + 1)
    return one(a) * one(b)


def test_plane_weights_exact_for_quadratics():
    for n, jitter in ((900, 0.0), (1500, 0.3)):
        surf = S.flat_square(n, L, np.random.default_rng(1), jitter)
        q, info = Q.plane_weights(surf.xyz, return_info=True)
        x, y = surf.xyz[:, 0], surf.xyz[:, 1]
        assert abs(info["area"] - L * L) < 1e-12 * L * L
        for a, b in ((0, 0), (1, 0), (0, 1), (2, 0), (1, 1), (0, 2)):
            exact = _square_monomial_integral(a, b)
            assert abs(q @ (x ** a * y ** b) - exact) <= 1e-12 * L ** (2 + a + b), (a, b)


def test_plane_weights_converge_for_smooth_integrand():
    exact = (6.0 * math.sinh(L / 6.0)) * (4.0 * math.sin(L / 4.0))
    errs = []
    for n in (1000, 4000):
        surf = S.flat_square(n, L)
        q = Q.plane_weights(surf.xyz)
        x, y = surf.xyz[:, 0], surf.xyz[:, 1]
        errs.append(abs(q @ (np.exp(x / 3.0) * np.cos(y / 2.0)) - exact) / abs(exact))
    assert errs[0] < 1e-5 and errs[1] < errs[0] / 16, errs


def test_flat_mms_nonlocal_term_matches_periodic_trapezoid():
    m = mms.FlatMMS(300)
    M = 160
    g = -L / 2 + L * np.arange(M) / M
    gx, gy = np.meshgrid(g, g, indexing="ij")
    grid = np.stack([gx.ravel(), gy.ravel(), np.zeros(M * M)], axis=1)
    t = 0.37
    X, Y, _, _ = m.centre(t)
    phi_grid = m.c0 + m.c1 * (1 + np.cos(grid[:, 0] - X)) * (1 + np.cos(grid[:, 1] - Y))
    rows = np.arange(0, m.surface.n, 7)
    pts = np.concatenate([m.surface.xyz[rows], grid])
    A_e, s_e, _, _ = m.kernel
    d = NF.distances(pts, np.arange(rows.size), L)[:, rows.size:]
    trap = (A_e * np.exp(-(d / s_e) ** 2)) @ phi_grid * (L / M) ** 2
    assert np.max(np.abs(trap - m.K_phi(t)[rows])) < 1e-12


def test_flat_mms_forcing_is_consistent():
    m = mms.FlatMMS(400)
    t, h = 0.05, 1e-5
    ut = (m.u(t + h) - m.u(t - h)) / (2 * h)
    F = m.forcing(t)
    assert np.max(np.abs(F - (ut + m.u(t) - m.K_phi(t)))) < 1e-8


def test_flat_mms_forced_system_converges():
    """Forced RK4 on the planar RBF-QF discretisation with the periodic kernel
    tracks the exact solution; the error falls >= 8x from N = 1000 to 4000."""
    errs = []
    dt, steps = 0.01, 10
    for n in (1000, 4000):
        m = mms.FlatMMS(n)
        q = Q.plane_weights(m.surface.xyz)
        op = NF.DenseOperator(m.surface.xyz, q, m.kind, m.kernel, period=L)
        F = m.stage_forcing(dt, steps)
        u = NF.rk4_forced(op, m.u(0.0)[None, :], m.beta, m.theta, dt, steps,
                          lambda k, c: F[k, {0.0: 0, 0.5: 1, 1.0: 2}[c]])
        ex = m.u(dt * steps)
        errs.append(np.max(np.abs(u[0] - ex)) / np.max(np.abs(ex)))
    assert errs[0] < 2e-4 and errs[1] < errs[0] / 8, errs


def test_periodic_adjoint_matches_finite_differences():
    rng = np.random.default_rng(2)
    surf = S.flat_square(200, L, rng, 0.3)
    q = Q.plane_weights(surf.xyz, k=16)
    p = (2.0, 0.6, 1.0, 1.5)
    u0 = rng.normal(0.5, 0.3, size=(1, surf.n))
    beta, theta, dt, steps = 5.0, 0.5, 0.05, 6
    target = rng.normal(0.5, 0.3, size=(1, surf.n))
    op = NF.ParamOperator(surf.xyz, q, NF.GAUSS_MH, p, period=L)
    _, gu, gp = NF.adjoint_gradients(op, u0, beta, theta, dt, steps, target)
    fd = NF.fd_param_gradients(surf.xyz, q, NF.GAUSS_MH, p, u0, beta, theta, dt, steps, target, h=1e-3, order=4,
                               period=L)
    assert np.max(np.abs(gp - fd) / np.maximum(np.abs(fd), 1e-3 * np.max(np.abs(fd)))) < 1e-6
    d = rng.normal(size=surf.n)
    d /= np.linalg.norm(d)
    fdu = NF.fd_u0_directional(surf.xyz, q, NF.GAUSS_MH, p, u0, beta, theta, dt, steps, target, d, h=1e-3,
                               order=4, period=L)
    assert abs(float(gu[0] @ d) - fdu) < 1e-7 * abs(fdu)
    # the periodic wrap matters here: the open-domain gradients differ
    op_open = NF.ParamOperator(surf.xyz, q, NF.GAUSS_MH, p)
    _, _, gp_open = NF.adjoint_gradients(op_open, u0, beta, theta, dt, steps, target)
    assert np.max(np.abs(gp_open - gp)) > 1e-3 * np.max(np.abs(gp))
