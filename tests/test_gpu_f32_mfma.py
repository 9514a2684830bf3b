"""GPU parity of the on-the-fly FP32 form with its products on the FP32 matrix
cores (ONTHEFLY_FP32_MFMA = 6).

Its arithmetic is that of the vector-unit FP32 form: kernel values in FP32,
FP32 products and FP32 sums over 256 sources folded into FP64 (the matrix
cores' FP32 products are those of an FMA), so the same tolerances apply:
|dy_i| <= 1e-5 S_i for one application (S_i = sum_j |w_ij q_j f(u_j)|) and
u(T) to 1e-5 relative L-infinity per state.
"""
import math

import numpy as np
import pytest
import torch

from oracle import neural_field as NF
from oracle import quadrature as Q
from workloads import configs as C
from workloads import surfaces as S

pytestmark = pytest.mark.gpu
P = pytest.importorskip("paper_2504_13379_amd")

FORM = 6
TOL = 1e-5
GAUSS = (1.0, 0.15, 0.5, 0.4)
EXPK = (2.0, 0.1, 1.0, 0.3)
L = 2.0 * math.pi


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return P.Context(0)


def _apply(ctx, x, q, U, kind, p, beta, theta, period=0.0, form=FORM):
    prob = P.Problem(ctx, torch.from_numpy(x).cuda(), torch.from_numpy(q).cuda(), period=period)
    k = P.kernel_struct(kind, *p)
    th = torch.from_numpy(np.asarray(theta, dtype=np.float64)).cuda() if np.ndim(theta) else float(theta)
    y = prob.apply(k, P.Firing(beta, th), torch.from_numpy(np.ascontiguousarray(U)).cuda(), form=form)
    torch.cuda.synchronize()
    return y.cpu().numpy()


def _scale(x, q, U, kind, p, beta, theta, rows=None, period=None):
    G = q[None, :] * NF.firing(U, beta, theta)
    return np.abs(G) @ np.abs(NF.kernel_matrix(x, kind, p, rows=rows, period=period)).T


@pytest.mark.parametrize("n,B", [(1, 1), (200, 3), (256, 32), (300, 33), (1000, 64), (2500, 70), (1100, 130)])
@pytest.mark.parametrize("kind", [NF.GAUSS_MH, NF.EXP_MH])
def test_f32_mfma_apply_matches_oracle(ctx, n, B, kind):
    rng = np.random.default_rng(11 * n + B + kind)
    x = S.fibonacci_sphere(n) * 1.05
    q = rng.uniform(0.5, 1.5, size=n) * 4 * math.pi / n
    if n > 3:
        q[rng.integers(n)] *= -0.1
    U = rng.normal(0.2, 0.4, size=(B, n))
    theta = rng.uniform(0.15, 0.3, size=B)
    p = GAUSS if kind == NF.GAUSS_MH else EXPK
    y = _apply(ctx, x, q, U, kind, p, 20.0, theta)
    ref = NF.apply_K(x, q, U, kind, p, 20.0, theta)
    err = np.max(np.abs(y - ref) / _scale(x, q, U, kind, p, 20.0, theta))
    assert err <= TOL, err


@pytest.mark.parametrize("kind,p", [(NF.GAUSS_MH, (1.0, 0.12, 0.4, 0.12 * math.sqrt(3.0))),   # rho = 1/3
                                    (NF.EXP_MH, (2.0, 0.1, 1.0, 0.4)),                        # rho = 1/4
                                    (NF.GAUSS_MH, (0.0, 0.15, 0.5, 0.4)),                     # no excitatory part
                                    (NF.GAUSS_MH, (-1.0, 0.15, 0.5, 0.4))])                   # negative A_e
def test_f32_mfma_kernel_variants(ctx, kind, p):
    n, B = 1500, 40
    rng = np.random.default_rng(n + int(1000 * abs(p[0])) + int(p[3] * 1000))
    x = S.fibonacci_sphere(n)
    q = rng.uniform(0.5, 1.5, size=n) * 4 * math.pi / n
    U = rng.normal(0.2, 0.4, size=(B, n))
    y = _apply(ctx, x, q, U, kind, p, 20.0, 0.2)
    ref = NF.apply_K(x, q, U, kind, p, 20.0, 0.2)
    assert np.max(np.abs(y - ref) / _scale(x, q, U, kind, p, 20.0, 0.2)) <= TOL


def test_f32_mfma_periodic_plane(ctx):
    """Doubly periodic square of side 2 pi (eq. dist), 8 states (scaled-period rounding as for the
    vector-unit form: within 1e-5)."""
    rng = np.random.default_rng(44)
    surf = S.flat_square(2000, L, rng, 0.3)
    q = Q.plane_weights(surf.xyz)
    B, p = 8, (1.0, 0.6, 0.5, 1.2)
    U = rng.normal(0.3, 0.4, size=(B, surf.n))
    theta = rng.uniform(0.1, 0.4, size=B)
    y = _apply(ctx, surf.xyz, q, U, NF.GAUSS_MH, p, 5.0, theta, period=L)
    ref = NF.apply_K(surf.xyz, q, U, NF.GAUSS_MH, p, 5.0, theta, period=L)
    assert np.max(np.abs(y - ref) / _scale(surf.xyz, q, U, NF.GAUSS_MH, p, 5.0, theta, period=L)) <= TOL


def test_f32_mfma_deterministic_and_close_to_vector_form(ctx):
    """Bitwise repeatable; against the vector-unit FP32 form the two differ only by the order of
    FP32 additions inside 256-source blocks (2 x 1e-5 bound)."""
    n, B = 2000, 64
    rng = np.random.default_rng(6)
    x = S.fibonacci_sphere(n)
    q = rng.uniform(0.5, 1.5, size=n) * 4 * math.pi / n
    U = rng.normal(0.2, 0.4, size=(B, n))
    theta = rng.uniform(0.15, 0.3, size=B)
    a = _apply(ctx, x, q, U, NF.GAUSS_MH, GAUSS, 20.0, theta)
    b = _apply(ctx, x, q, U, NF.GAUSS_MH, GAUSS, 20.0, theta)
    v = _apply(ctx, x, q, U, NF.GAUSS_MH, GAUSS, 20.0, theta, form=0)
    assert np.array_equal(a, b)
    assert np.max(np.abs(a - v) / _scale(x, q, U, NF.GAUSS_MH, GAUSS, 20.0, theta)) <= 2 * TOL


def test_f32_mfma_full_size_ellipsoid_sampled_rows(ctx):
    """Ellipsoid ensemble at its full size (N = 65536, B = 64): one application, sampled rows."""
    w = C.ellipsoid_ensemble()
    x = w.surface.xyz
    q = C.area_share_weights(w.surface)
    rows = np.random.default_rng(13).choice(w.n, 24, replace=False)
    y = _apply(ctx, x, q, w.u0, w.kernel_kind, w.kernel, w.beta, w.theta)
    ref = NF.apply_K(x, q, w.u0, w.kernel_kind, w.kernel, w.beta, w.theta, rows=rows)
    err = np.max(np.abs(y[:, rows] - ref) / _scale(x, q, w.u0, w.kernel_kind, w.kernel, w.beta, w.theta, rows))
    assert err <= TOL, err


@pytest.mark.parametrize("stepper", ["rk4", "rk4_graph", "ab5"])
def test_f32_mfma_integrate_ensemble_per_member(ctx, stepper):
    w = C.ellipsoid_ensemble(3000, 64, steps=30)
    q = Q.surface_weights(w.surface)
    op = NF.DenseOperator(w.surface.xyz, q, w.kernel_kind, w.kernel)
    c = P.Context(0, torch.cuda.Stream()) if stepper == "rk4_graph" else ctx
    prob = P.Problem(c, torch.from_numpy(w.surface.xyz).cuda(), torch.from_numpy(q).cuda())
    k = P.kernel_struct(w.kernel_kind, *w.kernel)
    f = P.Firing(w.beta, torch.from_numpy(w.theta).cuda())
    u = torch.from_numpy(w.u0.copy()).cuda()
    if stepper == "ab5":
        ref = NF.ab5(op, w.u0, w.beta, w.theta, w.dt, w.steps)
        prob.integrate_ab5(k, f, u, w.dt, w.steps, form=FORM)
    else:
        ref = NF.rk4(op, w.u0, w.beta, w.theta, w.dt, w.steps)
        prob.integrate(k, f, u, w.dt, w.steps, form=FORM, use_graph=stepper == "rk4_graph")
    torch.cuda.synchronize()
    err = NF.rel_linf(u.cpu().numpy(), ref)
    assert np.all(err <= TOL), err.max()


@pytest.mark.parametrize("B,expect", [(1, 0), (16, 0), (17, 6), (64, 6)])
def test_auto_form_picks_fp32_class_form(ctx, B, expect):
    """FORM_AUTO resolves to the FP32 matrix-core form above 16 states and to
    the vector-unit FP32 sum below: bitwise the result of that form."""
    n = 700
    rng = np.random.default_rng(90 + B)
    x = S.fibonacci_sphere(n)
    q = rng.uniform(0.5, 1.5, size=n) * 4 * math.pi / n
    U = rng.normal(0.2, 0.4, size=(B, n))
    prob = P.Problem(ctx, torch.from_numpy(x).cuda(), torch.from_numpy(q).cuda())
    k = P.kernel_struct(NF.GAUSS_MH, 1.0, 0.15, 0.5, 0.4)
    th = torch.from_numpy(rng.uniform(0.1, 0.3, size=B)).cuda() if B > 1 else 0.2
    f = P.Firing(20.0, th)
    u = torch.from_numpy(U).cuda()
    a = prob.apply(k, f, u, form=P.FORM_AUTO)
    b = prob.apply(k, f, u, form=expect)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
