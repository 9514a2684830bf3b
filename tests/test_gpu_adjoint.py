"""GPU adjoint (hand-written transpose pair sum + fused parameter gradients)
against the FP64 oracle's discrete adjoint, fourth-order finite differences,
and the beta = 0 closed forms.

Tolerance: the target for the adjoint is 1e-4 relative (norm-wise for the
u0-gradient, per parameter relative to max(|g_ref|, 1e-3 max|g_ref|) for the
five kernel/firing parameters).  The GPU trajectory carries FP32 pair sums
(relative ~1e-7 per application), which the adjoint inherits.
"""
import math
import os

import numpy as np
import pytest
import torch

from oracle import neural_field as NF
from oracle import quadrature as Q
from workloads import configs as C
from workloads import surfaces as S

pytestmark = pytest.mark.gpu
P = pytest.importorskip("paper_2504_13379_amd")
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "torus16384_adjoint.npz")
TOL = 1e-4


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return P.Context(0)


def _param_err(g, ref):
    floor = 1e-3 * np.max(np.abs(ref))
    return np.max(np.abs(g - ref) / np.maximum(np.abs(ref), floor))


def _gpu_grads(ctx, x, q, kind, p, u0, beta, theta, dt, steps, every, target):
    prob = P.Problem(ctx, torch.from_numpy(x).cuda(), torch.from_numpy(q).cuda())
    k = P.kernel_struct(kind, *p)
    f = P.Firing(beta, theta)
    u = torch.from_numpy(np.atleast_2d(u0).copy()).cuda()
    ck = prob.integrate(k, f, u, dt, steps, ckpt_every=every)
    uT = u.cpu().numpy()
    ubarT = torch.from_numpy(2.0 * (uT - target)).cuda()
    gu, gp = prob.adjoint(k, f, ck, every, steps, dt, ubarT)
    return uT, gu.cpu().numpy(), gp.numpy()


def _case(kind, n=700, steps=37, seed=3):
    rng = np.random.default_rng(seed)
    if kind == NF.EXP_MH:
        w = C.torus_exp(n, steps=steps, seed=seed)
    else:
        w = C.sphere_small(n)
        w.steps = steps
    q = Q.surface_weights(w.surface)
    tp = np.array(list(w.kernel) + [w.theta[0]]) * (1 + 0.05 * rng.uniform(-1, 1, size=5))
    target = NF.rk4(NF.DenseOperator(w.surface.xyz, q, w.kernel_kind, tp[:4]), w.u0, w.beta, tp[4], w.dt, steps)
    return w, q, target


@pytest.mark.parametrize("kind", [NF.EXP_MH, NF.GAUSS_MH])
def test_adjoint_matches_oracle_and_fd(ctx, kind):
    w, q, target = _case(kind)
    x, th = w.surface.xyz, float(w.theta[0])
    uT, gu, gp = _gpu_grads(ctx, x, q, w.kernel_kind, w.kernel, w.u0, w.beta, th, w.dt, w.steps, 10, target)
    op = NF.ParamOperator(x, q, w.kernel_kind, w.kernel)
    L, gu_ref, gp_ref = NF.adjoint_gradients(op, w.u0, w.beta, th, w.dt, w.steps, target)
    assert np.max(np.abs(gu - gu_ref[0])) <= TOL * np.max(np.abs(gu_ref))
    assert _param_err(gp, gp_ref) <= TOL
    fd = NF.fd_param_gradients(x, q, w.kernel_kind, w.kernel, w.u0, w.beta, th, w.dt, w.steps, target,
                               h=1e-3, order=4)
    assert _param_err(gp, fd) <= TOL
    d = np.random.default_rng(1).normal(size=w.n)
    d /= np.linalg.norm(d)
    fdu = NF.fd_u0_directional(x, q, w.kernel_kind, w.kernel, w.u0, w.beta, th, w.dt, w.steps, target, d,
                               h=1e-3, order=4)
    assert abs(float(gu @ d) - fdu) <= TOL * abs(fdu)


def test_adjoint_deterministic_and_autograd(ctx):
    w, q, target = _case(NF.EXP_MH, n=500, steps=12)
    x, th = w.surface.xyz, float(w.theta[0])
    a = _gpu_grads(ctx, x, q, w.kernel_kind, w.kernel, w.u0, w.beta, th, w.dt, w.steps, 5, target)
    b = _gpu_grads(ctx, x, q, w.kernel_kind, w.kernel, w.u0, w.beta, th, w.dt, w.steps, 5, target)
    assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
    prob = P.Problem(ctx, torch.from_numpy(x).cuda(), torch.from_numpy(q).cuda())
    u0 = torch.from_numpy(w.u0[0].copy()).cuda().requires_grad_(True)
    params = torch.tensor(list(w.kernel) + [th], dtype=torch.float64, requires_grad=True)
    uT = P.NeuralFieldRK4.apply(u0, params, prob, w.kernel_kind, w.beta, w.dt, w.steps, 5)
    loss = ((uT - torch.from_numpy(target[0]).cuda()) ** 2).sum()
    loss.backward()
    assert np.array_equal(u0.grad.cpu().numpy(), a[1])
    assert np.array_equal(params.grad.numpy(), a[2])


def test_adjoint_graph_replay_is_bitwise_eager():
    """On a context with its own stream the forward steps and the adjoint's segments
    replay captured graphs; the results equal the eagerly launched ones bit for bit
    (steps not a multiple of the checkpoint interval: two segment lengths)."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    w, q, target = _case(NF.EXP_MH, n=900, steps=23, seed=8)
    x, th = w.surface.xyz, float(w.theta[0])
    eager = _gpu_grads(P.Context(0), x, q, w.kernel_kind, w.kernel, w.u0, w.beta, th, w.dt, w.steps, 5, target)
    sctx = P.Context(0, torch.cuda.Stream())
    with torch.cuda.stream(sctx.stream):
        prob = P.Problem(sctx, torch.from_numpy(x).cuda(), torch.from_numpy(q).cuda())
        u0 = torch.from_numpy(w.u0[0].copy()).cuda().requires_grad_(True)
        params = torch.tensor(list(w.kernel) + [th], dtype=torch.float64, requires_grad=True)
        uT = P.NeuralFieldRK4.apply(u0, params, prob, w.kernel_kind, w.beta, w.dt, w.steps, 5)
        loss = ((uT - torch.from_numpy(target[0]).cuda()) ** 2).sum()
        loss.backward()
    torch.cuda.synchronize()
    assert np.array_equal(uT.detach().cpu().numpy(), eager[0][0])
    assert np.array_equal(u0.grad.cpu().numpy(), eager[1])
    assert np.array_equal(params.grad.numpy(), eager[2])


def test_adjoint_beta_zero_closed_form_full_size(ctx):
    """beta = 0 on the full-size torus adjoint workload (N = 16384): dL/du0 = R^n 2 (u(T) - target)
    and dL/dA_e = sum_i res_i (1 - R^n) / 2 sum_j exp(-r_ij / s_e) q_j."""
    w = C.torus_adjoint(16384, 60, ckpt_every=20)
    x = w.surface.xyz
    q = C.area_share_weights(w.surface)
    target = np.zeros((1, w.n))
    uT, gu, gp = _gpu_grads(ctx, x, q, w.kernel_kind, w.kernel, w.u0, 0.0, 0.25, w.dt, w.steps, 20, target)
    z = -w.dt
    R = (1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24) ** w.steps
    res = 2.0 * (uT[0] - target[0])
    assert np.max(np.abs(gu - R * res)) <= 1e-12 * np.max(np.abs(res))
    A_e, s_e, A_i, s_i = w.kernel
    rows = np.arange(w.n)
    ee = np.empty(w.n)
    for lo in range(0, w.n, 1024):
        d = np.sqrt(np.sum((x[lo:lo + 1024, None, :] - x[None, :, :]) ** 2, axis=2))
        ee[lo:lo + 1024] = np.exp(-d / s_e) @ q
    dAe = float(np.sum(res * (1 - R) * 0.5 * ee))
    assert abs(gp[0] - dAe) <= TOL * abs(dAe)
    assert abs(gp[4]) <= 1e-12 * np.max(np.abs(gp[:4]))


@pytest.mark.skipif(not os.path.exists(GOLDEN), reason="golden oracle adjoint not generated")
def test_adjoint_full_size_torus_against_oracle(ctx):
    """Torus adjoint workload at full size: N = 16384, 400 RK4 steps, checkpoints every 40."""
    g = np.load(GOLDEN)
    w = C.torus_adjoint(int(g["n"]), int(g["steps"]))
    uT, gu, gp = _gpu_grads(ctx, w.surface.xyz, g["q"], w.kernel_kind, w.kernel, w.u0, w.beta,
                            float(w.theta[0]), w.dt, w.steps, w.extra["ckpt_every"], g["target"])
    assert np.max(np.abs(uT - g["uT"])) <= 1e-5 * np.max(np.abs(g["uT"]))
    assert np.max(np.abs(gu - g["grad_u0"][0])) <= TOL * np.max(np.abs(g["grad_u0"]))
    assert _param_err(gp, g["grad_p"]) <= TOL


def test_central_fd_h1e4_through_gpu_forward(ctx):
    """Central differences with the absolute step h = 1e-4 taken through the GPU
    forward integration (five parameters and one unit u0 direction), on the
    torus with N = 700 nodes and 37 RK4 steps.

    FD(h) = (L(p + h) - L(p - h)) / 2h differs from the derivative by its
    truncation error, O(h^2) times the third derivative of L, which the steep
    sigmoid (beta = 20) can make visible; the FP64 oracle's FD with the same h
    carries the same truncation error.  The GPU's FD adds the rounding of its
    FP32 pair sums: the two losses carry independent errors
    dL ~ 2 |u - target| |du| with |du| ~ 1e-7 |u|, divided by 2h = 2e-4,
    about 1e-4 of the largest gradient component here (measured: 1.05e-4 for
    s_e; the oracle's FD and adjoint agree to 2e-6).  So, norm-wise against
    the largest component: the GPU's FD matches the oracle's FD, and the GPU
    adjoint matches the GPU's FD up to the oracle's own FD-versus-adjoint gap,
    both within 3e-4."""
    w, q, target = _case(NF.EXP_MH)
    x, th = w.surface.xyz, float(w.theta[0])
    h = 1e-4
    _, gu, gp = _gpu_grads(ctx, x, q, w.kernel_kind, w.kernel, w.u0, w.beta, th, w.dt, w.steps, 10, target)
    prob = P.Problem(ctx, torch.from_numpy(x).cuda(), torch.from_numpy(q).cuda())

    def loss_gpu(params, u0):
        u = torch.from_numpy(np.atleast_2d(u0).copy()).cuda()
        prob.integrate(P.kernel_struct(w.kernel_kind, *params[:4]), P.Firing(w.beta, float(params[4])), u, w.dt,
                       w.steps)
        torch.cuda.synchronize()
        return NF.loss(u.cpu().numpy(), target)
    base = np.array(list(w.kernel) + [th])
    fd_gpu = np.zeros(5)
    for m in range(5):
        e = np.zeros(5)
        e[m] = h
        fd_gpu[m] = (loss_gpu(base + e, w.u0) - loss_gpu(base - e, w.u0)) / (2 * h)
    fd_orc = NF.fd_param_gradients(x, q, w.kernel_kind, w.kernel, w.u0, w.beta, th, w.dt, w.steps, target, h=h)
    op = NF.ParamOperator(x, q, w.kernel_kind, w.kernel)
    _, gu_orc, gp_orc = NF.adjoint_gradients(op, w.u0, w.beta, th, w.dt, w.steps, target)
    print("fd_gpu", fd_gpu, "fd_orc", fd_orc, "adj_gpu", gp, "adj_orc", gp_orc, flush=True)
    scale = np.max(np.abs(fd_orc))
    assert np.max(np.abs(fd_gpu - fd_orc)) <= 3e-4 * scale
    trunc = np.abs(fd_orc - gp_orc)
    assert np.all(np.abs(fd_gpu - gp) <= trunc + 3e-4 * scale)
    d = np.random.default_rng(2).normal(size=w.n)
    d /= np.linalg.norm(d)
    fdu_gpu = (loss_gpu(base, w.u0 + h * d) - loss_gpu(base, w.u0 - h * d)) / (2 * h)
    fdu_orc = NF.fd_u0_directional(x, q, w.kernel_kind, w.kernel, w.u0, w.beta, th, w.dt, w.steps, target, d, h=h)
    print("u0 direction: fd_gpu %.8e fd_orc %.8e adj_gpu %.8e" % (fdu_gpu, fdu_orc, float(gu @ d)), flush=True)
    # the rounding allowance is absolute (dL / 2h), the same as for the parameters
    assert abs(fdu_gpu - fdu_orc) <= 3e-4 * scale
    assert abs(fdu_gpu - float(gu @ d)) <= abs(fdu_orc - float(gu_orc[0] @ d)) + 3e-4 * scale
