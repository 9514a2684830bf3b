"""GPU parity of the split-precision W forms on the matrix cores.

Tolerances from the arithmetic: W and f(u) are each carried as hi + 2^-c lo
(c = 8 for BF16, 11 for FP16), i.e. to a relative 2^-17 (BF16) or 2^-22
(FP16) per element, and the dropped lo*lo product is of the same order; with
FP32 accumulation a term of the sum is off by at most ~3e-5 (BF16) or ~1e-6
(FP16) of its magnitude.  One application is compared norm-wise against
S_i = sum_j |w_ij q_j f(u_j)|; u(T) to relative L-infinity 1e-4 (BF16, the
target for the split-BF16 form) and 1e-5 (FP16).
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

GAUSS = (1.0, 0.15, 0.5, 0.4)
EXPK = (2.0, 0.1, 1.0, 0.3)
TOL_APPLY = {2: 3e-5, 3: 2e-6}
TOL_STATE = {2: 1e-4, 3: 1e-5}


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return P.Context(0)


def _apply(ctx, x, q, U, kind, p, beta, theta, form):
    prob = P.Problem(ctx, torch.from_numpy(x).cuda(), torch.from_numpy(q).cuda())
    k = P.kernel_struct(kind, *p)
    th = torch.from_numpy(np.asarray(theta, dtype=np.float64)).cuda() if np.ndim(theta) else float(theta)
    W = prob.w_build(k, form)
    y = prob.apply(k, P.Firing(beta, th), torch.from_numpy(np.ascontiguousarray(U)).cuda(), form=form, W=W)
    torch.cuda.synchronize()
    return y.cpu().numpy()


def _scale(x, q, U, kind, p, beta, theta, rows=None):
    G = q[None, :] * NF.firing(U, beta, theta)
    return np.abs(G) @ np.abs(NF.kernel_matrix(x, kind, p, rows=rows)).T


@pytest.mark.parametrize("form", [2, 3])
@pytest.mark.parametrize("n,B", [(1, 1), (200, 3), (256, 32), (300, 33), (1000, 64), (2500, 70)])
@pytest.mark.parametrize("kind", [NF.GAUSS_MH, NF.EXP_MH])
def test_mfma_apply_matches_oracle(ctx, form, n, B, kind):
    rng = np.random.default_rng(7 * n + B + 100 * form + kind)
    x = S.fibonacci_sphere(n) * 1.05
    q = rng.uniform(0.5, 1.5, size=n) * 4 * math.pi / n
    U = rng.normal(0.2, 0.4, size=(B, n))
    theta = rng.uniform(0.15, 0.3, size=B)
    p = GAUSS if kind == NF.GAUSS_MH else EXPK
    y = _apply(ctx, x, q, U, kind, p, 20.0, theta, form)
    ref = NF.apply_K(x, q, U, kind, p, 20.0, theta)
    err = np.max(np.abs(y - ref) / _scale(x, q, U, kind, p, 20.0, theta))
    assert err <= TOL_APPLY[form], err


def test_mfma_fp16_scaling_handles_tiny_weights(ctx):
    """Weights ~1e-7 would underflow FP16 without the power-of-two lift of W."""
    n, B = 700, 8
    rng = np.random.default_rng(3)
    x = S.fibonacci_sphere(n)
    q = rng.uniform(0.5, 1.5, size=n) * 1e-7
    U = rng.normal(0.2, 0.4, size=(B, n))
    y = _apply(ctx, x, q, U, NF.GAUSS_MH, GAUSS, 20.0, 0.2, 3)
    ref = NF.apply_K(x, q, U, NF.GAUSS_MH, GAUSS, 20.0, 0.2)
    assert np.max(np.abs(y - ref) / _scale(x, q, U, NF.GAUSS_MH, GAUSS, 20.0, 0.2)) <= TOL_APPLY[3]


@pytest.mark.parametrize("form", [2, 3])
def test_mfma_full_size_ellipsoid_sampled_rows(ctx, form):
    """Ellipsoid ensemble at its full size (N = 65536, B = 64): one application, sampled rows."""
    w = C.ellipsoid_ensemble()
    x = w.surface.xyz
    q = C.area_share_weights(w.surface)
    rows = np.random.default_rng(11).choice(w.n, 24, replace=False)
    y = _apply(ctx, x, q, w.u0, w.kernel_kind, w.kernel, w.beta, w.theta, form)
    ref = NF.apply_K(x, q, w.u0, w.kernel_kind, w.kernel, w.beta, w.theta, rows=rows)
    err = np.max(np.abs(y[:, rows] - ref) / _scale(x, q, w.u0, w.kernel_kind, w.kernel, w.beta, w.theta, rows))
    print("split W form %d, N = %d, B = %d: one application, max |dy| / S over 24 rows = %.3e" % (form, w.n, w.b, err),
          flush=True)
    assert err <= TOL_APPLY[form], err


@pytest.fixture(scope="module")
def ensemble_case():
    w = C.ellipsoid_ensemble(3000, 64, steps=30)
    q = Q.surface_weights(w.surface)
    op = NF.DenseOperator(w.surface.xyz, q, w.kernel_kind, w.kernel)
    return w, q, NF.rk4(op, w.u0, w.beta, w.theta, w.dt, w.steps)


@pytest.mark.parametrize("form", [2, 3])
def test_mfma_integrate_ensemble_per_member(ctx, ensemble_case, form):
    w, q, ref = ensemble_case
    prob = P.Problem(ctx, torch.from_numpy(w.surface.xyz).cuda(), torch.from_numpy(q).cuda())
    k = P.kernel_struct(w.kernel_kind, *w.kernel)
    W = prob.w_build(k, form)
    u = torch.from_numpy(w.u0.copy()).cuda()
    prob.integrate(k, P.Firing(w.beta, torch.from_numpy(w.theta).cuda()), u, w.dt, w.steps, form=form, W=W)
    torch.cuda.synchronize()
    err = NF.rel_linf(u.cpu().numpy(), ref)
    assert err.shape == (64,)
    assert np.all(err <= TOL_STATE[form]), err.max()
