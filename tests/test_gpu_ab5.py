"""GPU Adams-Bashforth 5 stepper (the paper's section 5.1 integrator, RK4
start-up) against the FP64 oracle's AB5.  Tolerances as for RK4: u(T) to
relative L-infinity 1e-5 (FP32 and FP16x3 forms), 1e-4 (BF16x3), and for the
fused on-the-fly split forms 1e-4 (BF16) and 2e-5 (FP16) as derived in
test_gpu_mfma_otf."""
import numpy as np
import pytest
import torch

from oracle import neural_field as NF
from oracle import quadrature as Q
from workloads import configs as C

pytestmark = pytest.mark.gpu
P = pytest.importorskip("paper_2504_13379_amd")
TOL = {0: 1e-5, 1: 1e-5, 2: 1e-4, 3: 1e-5, 4: 1e-4, 5: 2e-5, 6: 1e-5}


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return P.Context(0)


@pytest.mark.parametrize("form", [0, 1])
@pytest.mark.parametrize("steps", [3, 5, 120])
def test_ab5_sphere_single_state(ctx, form, steps):
    w = C.sphere_small()
    q = Q.surface_weights(w.surface)
    dt = 0.02
    ref = NF.ab5(NF.DenseOperator(w.surface.xyz, q, w.kernel_kind, w.kernel), w.u0, w.beta, w.theta, dt, steps)
    prob = P.Problem(ctx, torch.from_numpy(w.surface.xyz).cuda(), torch.from_numpy(q).cuda())
    k = P.kernel_struct(w.kernel_kind, *w.kernel)
    W = prob.w_build(k, form) if form else None
    u = torch.from_numpy(w.u0.copy()).cuda()
    prob.integrate_ab5(k, P.Firing(w.beta, float(w.theta[0])), u, dt, steps, form=form, W=W)
    torch.cuda.synchronize()
    assert np.all(NF.rel_linf(u.cpu().numpy(), ref) <= TOL[form])


@pytest.mark.parametrize("form,B", [(0, 6), (2, 6), (3, 6), (4, 6), (5, 6), (6, 6), (4, 40), (5, 40)])
def test_ab5_ensemble(ctx, form, B):
    # B = 40: the fused forms' 64-state kernels (for BF16 the eight-wave far form)
    w = C.ellipsoid_ensemble(2500, B, steps=40)
    q = Q.surface_weights(w.surface)
    ref = NF.ab5(NF.DenseOperator(w.surface.xyz, q, w.kernel_kind, w.kernel), w.u0, w.beta, w.theta, w.dt, w.steps)
    prob = P.Problem(ctx, torch.from_numpy(w.surface.xyz).cuda(), torch.from_numpy(q).cuda())
    k = P.kernel_struct(w.kernel_kind, *w.kernel)
    W = prob.w_build(k, form) if form in (1, 2, 3) else None
    u = torch.from_numpy(w.u0.copy()).cuda()
    prob.integrate_ab5(k, P.Firing(w.beta, torch.from_numpy(w.theta).cuda()), u, w.dt, w.steps, form=form, W=W)
    torch.cuda.synchronize()
    assert np.all(NF.rel_linf(u.cpu().numpy(), ref) <= TOL[form])


def test_ab5_first_four_steps_equal_rk4(ctx):
    w = C.sphere_small(700)
    q = C.area_share_weights(w.surface)
    prob = P.Problem(ctx, torch.from_numpy(w.surface.xyz).cuda(), torch.from_numpy(q).cuda())
    k = P.kernel_struct(w.kernel_kind, *w.kernel)
    f = P.Firing(w.beta, float(w.theta[0]))
    a = torch.from_numpy(w.u0.copy()).cuda()
    b = torch.from_numpy(w.u0.copy()).cuda()
    prob.integrate_ab5(k, f, a, 0.05, 4)
    prob.integrate(k, f, b, 0.05, 4)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
