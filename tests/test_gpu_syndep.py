"""GPU neural field with synaptic depression (paper section 5.2, eq. nfsyndep)
against the FP64 oracle; u(T) and a(T) to relative L-infinity 1e-5 per state."""
import numpy as np
import pytest
import torch

from oracle import neural_field as NF
from oracle import quadrature as Q
from workloads import configs as C

pytestmark = pytest.mark.gpu
P = pytest.importorskip("paper_2504_13379_amd")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return P.Context(0)


@pytest.mark.parametrize("B", [1, 3])
def test_syndep_matches_oracle(ctx, B):
    w = C.bumpy_syndep(3000, steps=40)
    q = Q.surface_weights(w.surface)
    rng = np.random.default_rng(B)
    u0 = np.repeat(w.u0, B, axis=0) + rng.normal(0, 0.01, size=(B, w.n))
    a0 = rng.uniform(0.6, 1.0, size=(B, w.n))
    theta = np.full(B, 0.3)
    tau, bd = w.extra["tau"], w.extra["beta_d"]
    op = NF.DenseOperator(w.surface.xyz, q, w.kernel_kind, w.kernel)
    ur, ar = NF.syndep_rk4(op, u0, a0, w.beta, theta, tau, bd, w.dt, w.steps)
    prob = P.Problem(ctx, torch.from_numpy(w.surface.xyz).cuda(), torch.from_numpy(q).cuda())
    u = torch.from_numpy(u0.copy()).cuda()
    a = torch.from_numpy(a0.copy()).cuda()
    prob.integrate_syndep(P.kernel_struct(w.kernel_kind, *w.kernel), P.Firing(w.beta, 0.3), u, a, tau, bd, w.dt,
                          w.steps)
    torch.cuda.synchronize()
    assert np.all(NF.rel_linf(u.cpu().numpy(), ur) <= 1e-5)
    assert np.all(NF.rel_linf(a.cpu().numpy(), ar) <= 1e-5)


def test_syndep_without_depression_equals_plain_integration(ctx):
    w = C.sphere_small(900)
    q = C.area_share_weights(w.surface)
    prob = P.Problem(ctx, torch.from_numpy(w.surface.xyz).cuda(), torch.from_numpy(q).cuda())
    k = P.kernel_struct(w.kernel_kind, *w.kernel)
    f = P.Firing(w.beta, float(w.theta[0]))
    u1 = torch.from_numpy(w.u0.copy()).cuda()
    a1 = torch.ones_like(u1)
    prob.integrate_syndep(k, f, u1, a1, 10.0, 0.0, 0.05, 12)
    u2 = torch.from_numpy(w.u0.copy()).cuda()
    prob.integrate(k, f, u2, 0.05, 12)
    torch.cuda.synchronize()
    assert torch.equal(a1, torch.ones_like(a1))
    assert torch.equal(u1, u2)
