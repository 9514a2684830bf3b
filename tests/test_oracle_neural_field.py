"""Pins for the oracle's operator, RK4 integrator and discrete adjoint (CPU only).

* the dense pair sum against brute force with exactly rounded sums (math.fsum);
* row sums on the sphere against the closed-form kernel integral;
* beta = 0 (f = 1/2): the RK4 solution, its u0-gradient and its A_e/s_e
  gradients in closed form through the RK4 stability polynomial;
* time convergence: halving dt cuts the error 16x, against scipy's DOP853;
* discrete adjoint against fourth-order finite differences with a step sweep.
"""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle import neural_field as NF
from oracle import quadrature as Q
from tests import pins
from workloads import configs as C
from workloads import surfaces as S

GAUSS = (1.0, 0.15, 0.5, 0.4)
EXPK = (2.0, 0.1, 1.0, 0.3)


def _problem(n=30, seed=0, kind=NF.GAUSS_MH):
    rng = np.random.default_rng(seed)
    x = S.fibonacci_sphere(n)
    q = rng.uniform(0.5, 1.5, size=n) * 4 * math.pi / n
    q[3] = -0.1 * q[3]                              # one small negative weight, as RBF-QF can give
    U = rng.normal(0.2, 0.5, size=(2, n))
    return x, q, U, (GAUSS if kind == NF.GAUSS_MH else EXPK)


@pytest.mark.parametrize("kind", [NF.GAUSS_MH, NF.EXP_MH])
def test_pair_sum_matches_bruteforce(kind):
    x, q, U, p = _problem(kind=kind)
    beta, theta = 20.0, np.array([0.2, 0.3])
    got = NF.apply_K(x, q, U, kind, p, beta, theta)
    n = x.shape[0]
    A_e, s_e, A_i, s_i = p
    for b in range(2):
        for i in range(n):
            terms = []
            for j in range(n):
                r = math.sqrt(sum((x[i][c] - x[j][c]) ** 2 for c in range(3)))
                if kind == NF.GAUSS_MH:
                    w = A_e * math.exp(-(r / s_e) ** 2) - A_i * math.exp(-(r / s_i) ** 2)
                else:
                    w = A_e * math.exp(-r / s_e) - A_i * math.exp(-r / s_i)
                f = 1.0 / (1.0 + math.exp(-beta * (U[b, j] - theta[b])))
                terms.append(w * q[j] * f)
            assert abs(got[b, i] - math.fsum(terms)) <= 1e-13 * max(1.0, sum(abs(t) for t in terms))
    op = NF.DenseOperator(x, q, kind, p)
    np.testing.assert_allclose(op.K(U, beta, theta), got, rtol=1e-13, atol=1e-15)
    rows = np.array([5, 0, 17])
    np.testing.assert_allclose(NF.apply_K(x, q, U, kind, p, beta, theta, rows=rows), got[:, rows],
                               rtol=1e-13, atol=1e-15)


def test_self_pair_is_included():
    x = np.array([[0.0, 0, 1], [0.0, 0, -1]])     # far apart: w(2) negligible
    q = np.array([0.5, 0.5])
    U = np.array([[50.0, 50.0]])                  # f = 1
    y = NF.apply_K(x, q, U, NF.EXP_MH, EXPK, 20.0, 0.25)
    w0 = EXPK[0] - EXPK[2]
    w2 = EXPK[0] * math.exp(-2 / EXPK[1]) - EXPK[2] * math.exp(-2 / EXPK[3])
    np.testing.assert_allclose(y, [[0.5 * (w0 + w2)] * 2], rtol=1e-14)


@pytest.fixture(scope="module")
def sphere_rules():
    out = {}
    for n in (4000, 16000):
        s = S.sphere(n)
        out[n] = (s, Q.surface_weights(s))
    return out


def _row_sum_error(rule, kind, p):
    s, q = rule
    n = s.n
    rows = np.arange(0, n, n // 40)
    big = 100.0                                    # f = 1 everywhere -> K_i = sum_j w_ij q_j
    y = NF.apply_K(s.xyz, q, np.full((1, n), big), kind, p, 20.0, 0.0, rows=rows)[0]
    return np.max(np.abs(y - pins.sphere_kernel_integral(kind, p)))


def test_sphere_row_sums_match_closed_form_gauss(sphere_rules):
    scale = pins.sphere_kernel_integral(NF.GAUSS_MH, (GAUSS[0], GAUSS[1], 0.0, GAUSS[3]))
    assert _row_sum_error(sphere_rules[4000], NF.GAUSS_MH, GAUSS) < 2e-4 * abs(scale)


def test_sphere_row_sums_converge_exp(sphere_rules):
    # the exponential kernel has a derivative jump at r = 0; its row sums still converge
    e1 = _row_sum_error(sphere_rules[4000], NF.EXP_MH, EXPK)
    e2 = _row_sum_error(sphere_rules[16000], NF.EXP_MH, EXPK)
    scale = pins.sphere_kernel_integral(NF.EXP_MH, (EXPK[0], EXPK[1], 0.0, EXPK[3]))
    assert e2 < e1 / 4 and e2 < 1e-3 * abs(scale)


def test_rk4_beta_zero_closed_form():
    x, q, U, p = _problem(n=40, seed=1, kind=NF.EXP_MH)
    op = NF.DenseOperator(x, q, NF.EXP_MH, p)
    dt, steps = 0.05, 37
    uT = NF.rk4(op, U, 0.0, 0.3, dt, steps)
    b = 0.5 * (op.w @ q)
    R = pins.rk4_amplification(-dt) ** steps
    np.testing.assert_allclose(uT, b + R * (U - b), rtol=1e-12, atol=1e-13)


def test_rk4_fourth_order_against_dop853():
    s = S.sphere(150)
    q = np.full(150, 4 * math.pi / 150)
    op = NF.DenseOperator(s.xyz, q, NF.GAUSS_MH, GAUSS)
    rng = np.random.default_rng(5)
    u0 = C.bump(s.xyz, s.xyz[7])[None, :] + rng.normal(0, 0.01, size=(1, 150))
    T = 2.0
    ref = solve_ivp(NF.rk4_rhs_dense(op, 20.0, 0.2), (0, T), u0.ravel(), method="DOP853",
                    rtol=1e-13, atol=1e-13).y[:, -1]
    errs = []
    for dt in (0.1, 0.05, 0.025):
        uT = NF.rk4(op, u0, 20.0, 0.2, dt, int(round(T / dt)))
        errs.append(np.max(np.abs(uT.ravel() - ref)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 13 < r1 < 19 and 13 < r2 < 19


def _adjoint_case(n=120, steps=12, kind=NF.EXP_MH, beta=20.0, seed=2):
    rng = np.random.default_rng(seed)
    surf = S.torus(n, rng) if kind == NF.EXP_MH else S.sphere(n)
    q = np.full(n, C.surface_area(surf) / n) * rng.uniform(0.8, 1.2, size=n)
    p = EXPK if kind == NF.EXP_MH else GAUSS
    u0 = (C.bump(surf.xyz, surf.xyz[3]) + C.bump(surf.xyz, surf.xyz[n // 2]))[None, :]
    tp = np.array(list(p) + [0.25]) * (1 + 0.05 * rng.uniform(-1, 1, size=5))
    target = NF.rk4(NF.DenseOperator(surf.xyz, q, kind, tp[:4]), u0, beta, tp[4], 0.02, steps)
    return surf.xyz, q, p, u0, beta, 0.25, 0.02, steps, target


@pytest.mark.parametrize("kind", [NF.EXP_MH, NF.GAUSS_MH])
def test_adjoint_matches_fourth_order_fd(kind):
    x, q, p, u0, beta, theta, dt, steps, target = _adjoint_case(kind=kind)
    op = NF.ParamOperator(x, q, kind, p)
    L, gu, gp = NF.adjoint_gradients(op, u0, beta, theta, dt, steps, target)
    assert L == pytest.approx(NF.loss(NF.rk4(op, u0, beta, theta, dt, steps), target), rel=1e-14)
    fd3 = NF.fd_param_gradients(x, q, kind, p, u0, beta, theta, dt, steps, target, h=1e-3, order=4)
    fd4 = NF.fd_param_gradients(x, q, kind, p, u0, beta, theta, dt, steps, target, h=1e-4, order=4)
    # the step sweep shows FD itself has converged where it is compared
    conv = np.abs(fd3 - fd4) / np.abs(fd4)
    assert np.all(conv < 1e-6)
    np.testing.assert_allclose(gp, fd4, rtol=1e-7)
    d = np.random.default_rng(9).normal(size=x.shape[0])
    d /= np.linalg.norm(d)
    fdu = NF.fd_u0_directional(x, q, kind, p, u0, beta, theta, dt, steps, target, d, h=1e-3, order=4)
    assert float(np.sum(gu * d)) == pytest.approx(fdu, rel=1e-7, abs=1e-14)


def test_adjoint_beta_zero_closed_forms():
    x, q, p, u0, _, theta, dt, steps, target = _adjoint_case(n=60, steps=15)
    op = NF.ParamOperator(x, q, NF.EXP_MH, p)
    L, gu, gp = NF.adjoint_gradients(op, u0, 0.0, theta, dt, steps, target)
    R = pins.rk4_amplification(-dt) ** steps
    A_e, s_e, A_i, s_i = p
    r = np.sqrt(np.sum((x[:, None, :] - x[None, :, :]) ** 2, axis=2))
    b = 0.5 * (A_e * np.exp(-r / s_e) - A_i * np.exp(-r / s_i)) @ q
    uT = b + R * (u0 - b)
    res = 2 * (uT - target)
    np.testing.assert_allclose(gu, R * res, rtol=1e-11, atol=1e-16)
    dAe = (1 - R) * 0.5 * (np.exp(-r / s_e) @ q)
    dse = (1 - R) * 0.5 * ((A_e * np.exp(-r / s_e) * r / s_e ** 2) @ q)
    dAi = -(1 - R) * 0.5 * (np.exp(-r / s_i) @ q)
    np.testing.assert_allclose(gp[0], float(np.sum(res * dAe)), rtol=1e-11)
    np.testing.assert_allclose(gp[1], float(np.sum(res * dse)), rtol=1e-11)
    np.testing.assert_allclose(gp[2], float(np.sum(res * dAi)), rtol=1e-11)
    assert abs(gp[4]) < 1e-15                       # f does not depend on theta when beta = 0


def test_fd_step_1e4_second_order_is_truncation_limited():
    """Plain central FD at h = 1e-4 agrees with the adjoint norm-wise to 1e-4; what is
    left over per component is FD truncation (it shrinks 100x when h shrinks 10x)."""
    x, q, p, u0, beta, theta, dt, steps, target = _adjoint_case(n=80, steps=10)
    op = NF.ParamOperator(x, q, NF.EXP_MH, p)
    _, _, gp = NF.adjoint_gradients(op, u0, beta, theta, dt, steps, target)
    fd2 = NF.fd_param_gradients(x, q, NF.EXP_MH, p, u0, beta, theta, dt, steps, target, h=1e-4)
    assert np.max(np.abs(fd2 - gp)) <= 1e-4 * np.max(np.abs(gp))
    fd2b = NF.fd_param_gradients(x, q, NF.EXP_MH, p, u0, beta, theta, dt, steps, target, h=1e-3)
    worst = np.argmax(np.abs(fd2 - gp) / np.abs(gp))
    ratio = abs(fd2b[worst] - gp[worst]) / abs(fd2[worst] - gp[worst])
    assert 50 < ratio < 200


def test_ab5_weights_integrate_the_interpolating_polynomial():
    """a_k = int_0^1 L_k(s) ds with L_k the Lagrange basis on the nodes s = 0, -1, ..., -4
    (the defining property of Adams-Bashforth weights), in exact rational arithmetic."""
    from fractions import Fraction
    nodes = [0, -1, -2, -3, -4]
    for k, a in enumerate(NF.AB5_WEIGHTS):
        poly = [Fraction(1)]                       # coefficients, lowest degree first
        denom = Fraction(1)
        for m, sm in enumerate(nodes):
            if m == k:
                continue
            poly = [Fraction(0)] + poly            # multiply by s
            for d in range(len(poly) - 1):
                poly[d] -= sm * poly[d + 1]        # ... minus s_m
            denom *= nodes[k] - sm
        integral = sum(c / (d + 1) for d, c in enumerate(poly)) / denom
        assert abs(float(integral) - a) < 1e-15


def test_ab5_fifth_order_against_dop853():
    s = S.sphere(120)
    q = np.full(120, 4 * math.pi / 120)
    op = NF.DenseOperator(s.xyz, q, NF.GAUSS_MH, GAUSS)
    u0 = C.bump(s.xyz, s.xyz[5])[None, :]
    T = 2.0
    ref = solve_ivp(NF.rk4_rhs_dense(op, 20.0, 0.2), (0, T), u0.ravel(), method="DOP853",
                    rtol=1e-13, atol=1e-13).y[:, -1]
    errs = [np.max(np.abs(NF.ab5(op, u0, 20.0, 0.2, dt, int(round(T / dt))).ravel() - ref))
            for dt in (0.04, 0.02, 0.01)]
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 24 < r1 < 40 and 24 < r2 < 40, (r1, r2)


def test_ab5_beta_zero_matches_companion_matrix():
    """beta = 0: e_n = u_n - b obeys e_{n+1} = e_n - dt sum_k a_k e_{n-k} after an RK4 start;
    the state after n steps is a power of the 5 x 5 companion matrix applied to the start."""
    x, q, U, p = _problem(n=25, seed=4, kind=NF.EXP_MH)
    op = NF.DenseOperator(x, q, NF.EXP_MH, p)
    dt, steps = 0.05, 23
    b = 0.5 * (op.w @ q)
    R = pins.rk4_amplification(-dt)
    e0 = U[0] - b
    start = [R ** n * e0 for n in range(5)]        # e_0 .. e_4 from the RK4 start
    Cm = np.zeros((5, 5))
    Cm[0, 0] = 1 - dt * NF.AB5_WEIGHTS[0]
    Cm[0, 1:] = [-dt * a for a in NF.AB5_WEIGHTS[1:]]
    Cm[1:, :4] = np.eye(4)
    state = np.stack(start[::-1])                  # rows: e_4, e_3, ..., e_0
    state = np.linalg.matrix_power(Cm, steps - 4) @ state
    got = NF.ab5(op, U[:1], 0.0, 0.3, dt, steps)[0]
    np.testing.assert_allclose(got, b + state[0], rtol=1e-11, atol=1e-13)


def test_syndep_without_depression_reduces_to_plain_model():
    """beta_d = 0 and a(0) = 1: the efficacy stays 1 and u follows the plain RK4 exactly."""
    x, q, U, p = _problem(n=35, seed=6)
    op = NF.DenseOperator(x, q, NF.GAUSS_MH, p)
    u, a = NF.syndep_rk4(op, U, np.ones_like(U), 20.0, np.array([0.2, 0.3]), 20.0, 0.0, 0.05, 17)
    np.testing.assert_array_equal(a, np.ones_like(U))
    np.testing.assert_allclose(u, NF.rk4(op, U, 20.0, np.array([0.2, 0.3]), 0.05, 17), rtol=1e-14, atol=1e-15)


def test_syndep_efficacy_closed_form_at_beta_zero():
    """beta = 0 (f = 1/2): tau a' = 1 - a (1 + beta_d/2), so the RK4 efficacy is
    a_n = a* + R(-dt (1 + beta_d/2) / tau)^n (a0 - a*),  a* = 1 / (1 + beta_d/2)."""
    x, q, U, p = _problem(n=20, seed=7)
    op = NF.DenseOperator(x, q, NF.EXP_MH, EXPK)
    rng = np.random.default_rng(1)
    a0 = rng.uniform(0.2, 1.0, size=U.shape)
    tau, bd, dt, n = 15.0, 1.3, 0.1, 31
    _, a = NF.syndep_rk4(op, U, a0, 0.0, 0.2, tau, bd, dt, n)
    astar = 1.0 / (1.0 + bd / 2.0)
    R = pins.rk4_amplification(-dt * (1.0 + bd / 2.0) / tau)
    np.testing.assert_allclose(a, astar + R ** n * (a0 - astar), rtol=1e-13)


def test_syndep_fourth_order_against_dop853():
    s = S.bumpy_sphere(140)
    q = np.full(140, 4 * math.pi / 140)
    op = NF.DenseOperator(s.xyz, q, NF.GAUSS_MH, GAUSS)
    u0 = C.bump(s.xyz, s.xyz[9])[None, :]
    a0 = np.full_like(u0, 0.9)
    beta, theta, tau, bd = 20.0, 0.2, 5.0, 2.0

    def fun(_t, y):
        du, da = NF.syndep_rhs(op, y[:140][None, :], y[140:][None, :], beta, theta, tau, bd)
        return np.concatenate([du.ravel(), da.ravel()])
    T = 2.0
    ref = solve_ivp(fun, (0, T), np.concatenate([u0.ravel(), a0.ravel()]), method="DOP853",
                    rtol=1e-13, atol=1e-13).y[:, -1]
    errs = []
    for dt in (0.1, 0.05, 0.025):
        u, a = NF.syndep_rk4(op, u0, a0, beta, theta, tau, bd, dt, int(round(T / dt)))
        errs.append(np.max(np.abs(np.concatenate([u.ravel(), a.ravel()]) - ref)))
    assert 13 < errs[0] / errs[1] < 19 and 13 < errs[1] / errs[2] < 19


def test_funk_hecke_constant_matches_closed_form():
    from workloads import mms
    for kind, p in ((NF.GAUSS_MH, GAUSS), (NF.EXP_MH, EXPK)):
        assert abs(mms.funk_hecke(kind, p, 0) - pins.sphere_kernel_integral(kind, p)) < 1e-11


def test_manufactured_solution_converges_with_quadrature():
    """The forced discrete system reproduces the manufactured solution; its error
    (quadrature of the operator + RK4) falls >= 4x from N = 1000 to 4000."""
    from workloads import mms
    errs = []
    for n in (1000, 4000):
        m = mms.SphereMMS(n)
        q = Q.surface_weights(m.surface)
        op = NF.DenseOperator(m.surface.xyz, q, m.kind, m.kernel)
        dt, steps = 0.02, 25
        F = m.stage_forcing(dt, steps)
        u = NF.rk4_forced(op, m.u(0.0)[None, :], m.beta, m.theta, dt, steps,
                          lambda k, c: F[k, {0.0: 0, 0.5: 1, 1.0: 2}[c]])
        errs.append(np.max(np.abs(u[0] - m.u(dt * steps))) / np.max(np.abs(m.u(dt * steps))))
    assert errs[1] < errs[0] / 4 and errs[1] < 1e-5, errs


def test_far_block_threshold_drops_steep_term_in_fp32():
    """The fused BF16 form evaluates only the broad exponential for pairs with
    (1 - rho) t > 27 - log2|kappa| (t = r^2 log2(e) / s_e^2, rho = s_e^2 / s_i^2,
    kappa = -A_i / A_e).  There the steep term 2^-t is below an eighth of a unit
    in the last place of the FP32 value kappa 2^(-rho t), so the FP32 sum equals
    the broad term alone: checked in FP32 arithmetic for several kernels."""
    rng = np.random.default_rng(0)
    for kappa in (-0.5, -1e-3, -3.0, 0.25, -2.0 ** -20):
        for rho in (0.1, 0.140625, 0.5, 0.75):
            tmin = (27.0 - np.log2(abs(kappa))) / (1.0 - rho)
            t = tmin * (1.0 + rng.uniform(0.0, 3.0, size=20000)) + 1e-9
            broad = (kappa * np.exp2(-rho * t)).astype(np.float32)
            steep = np.exp2(-t)
            total = (broad.astype(np.float64) + steep).astype(np.float32)
            assert np.array_equal(total, broad), (kappa, rho)
            ulp = np.spacing(np.abs(broad)).astype(np.float64)
            assert np.all(steep < ulp / 8), (kappa, rho)
