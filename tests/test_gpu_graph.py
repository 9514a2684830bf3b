"""Graph replay of nfr_integrate: groups of up to 64 RK4 steps captured once
into one HIP graph, kept with the problem and replayed by later calls with the
same arguments.  Every replayed result must equal the directly launched one
bit for bit (the same kernels with the same plan), including step counts that
are not a multiple of the group length, checkpoints (groups divide the
checkpoint interval), a changed argument (the graph is recaptured) and the
multi-state and matrix-core forms.  Against the oracle at the end.
"""
import ctypes

import numpy as np
import pytest
import torch

from oracle import neural_field as NF
from oracle import quadrature as Q
from workloads import configs as C

pytestmark = pytest.mark.gpu
P = pytest.importorskip("paper_2504_13379_amd")


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = P.Context(0, torch.cuda.Stream())
    w = C.sphere_small(2000)
    q = Q.surface_weights(w.surface)
    prob = P.Problem(ctx, torch.from_numpy(w.surface.xyz).cuda(), torch.from_numpy(q).cuda())
    return ctx, w, q, prob


def _run(ctx, prob, k, f, u0, dt, steps, graph, form=0, ckpt_every=0, B=1):
    u = torch.from_numpy(np.ascontiguousarray(u0)).cuda()
    ws = prob.integrate_workspace(B, form)
    ck = prob.integrate(k, f, u, dt, steps, form=form, ckpt_every=ckpt_every, use_graph=graph, ws=ws)
    ctx.stream.synchronize()
    return u.cpu().numpy(), (None if ck is None else ck.cpu().numpy()), ws


def _last_graph(ctx):
    nodes, steps = ctypes.c_int64(), ctypes.c_int64()
    P._lib.check(P.lib().nfr_context_last_graph(ctx.handle, ctypes.byref(nodes), ctypes.byref(steps)))
    return nodes.value, steps.value


def test_multi_step_graph_equals_launched(setup):
    ctx, w, q, prob = setup
    k = P.kernel_struct(w.kernel_kind, *w.kernel)
    f = P.Firing(w.beta, float(w.theta[0]))
    for steps in (150, 64, 7):
        a, _, _ = _run(ctx, prob, k, f, w.u0, w.dt, steps, False)
        g, _, _ = _run(ctx, prob, k, f, w.u0, w.dt, steps, True)
        assert np.array_equal(a, g), steps
        nodes, gsteps = _last_graph(ctx)
        assert gsteps == min(steps, 64)
        # small single-state problems: one launch per RK4 stage
        assert nodes == 4 * gsteps, (nodes, gsteps)
    ref = NF.rk4(NF.DenseOperator(w.surface.xyz, q, w.kernel_kind, w.kernel), w.u0, w.beta, w.theta, w.dt, 150)
    a, _, _ = _run(ctx, prob, k, f, w.u0, w.dt, 150, True)
    assert NF.rel_linf(a, ref).max() <= 1e-5


def test_graph_reused_and_recaptured(setup):
    """Two calls with the same arguments and workspace reuse the captured graph;
    a changed step size or kernel parameter is captured afresh (stale kernel
    arguments would show as a wrong result)."""
    ctx, w, q, prob = setup
    k = P.kernel_struct(w.kernel_kind, *w.kernel)
    f = P.Firing(w.beta, float(w.theta[0]))
    u = torch.from_numpy(w.u0.copy()).cuda()
    ws = prob.integrate_workspace(1, 0)
    outs = []
    for dt, kern in ((0.05, w.kernel), (0.05, w.kernel), (0.03, w.kernel), (0.03, (1.1, 0.15, 0.5, 0.4))):
        u.copy_(torch.from_numpy(w.u0))
        prob.integrate(P.kernel_struct(w.kernel_kind, *kern), f, u, dt, 40, use_graph=True, ws=ws)
        ctx.stream.synchronize()
        got = u.cpu().numpy()
        ref, _, _ = _run(ctx, prob, P.kernel_struct(w.kernel_kind, *kern), f, w.u0, dt, 40, False)
        assert np.array_equal(got, ref), (dt, kern)
        outs.append(got)
    assert np.array_equal(outs[0], outs[1])
    assert not np.array_equal(outs[1], outs[2]) and not np.array_equal(outs[2], outs[3])


@pytest.mark.parametrize("every,steps", [(10, 35), (40, 40), (96, 200), (7, 30)])
def test_graph_checkpoints(setup, every, steps):
    ctx, w, q, prob = setup
    k = P.kernel_struct(w.kernel_kind, *w.kernel)
    f = P.Firing(w.beta, float(w.theta[0]))
    a, cka, _ = _run(ctx, prob, k, f, w.u0, w.dt, steps, False, ckpt_every=every)
    g, ckg, _ = _run(ctx, prob, k, f, w.u0, w.dt, steps, True, ckpt_every=every)
    assert np.array_equal(a, g)
    assert cka.shape == (1 + steps // every, 1, w.n)
    assert np.array_equal(cka, ckg)
    _, gsteps = _last_graph(ctx)
    assert every % gsteps == 0 and gsteps <= 64


@pytest.mark.parametrize("form,B", [(0, 4), (6, 32), (4, 64), (0, 1)])
def test_graph_multi_state_forms(form, B):
    """Multi-state and matrix-core forms, and a single state on the symmetric
    (large-problem) kernel, replayed from multi-step graphs."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = P.Context(0, torch.cuda.Stream())
    w = C.ellipsoid_ensemble(5000 if B > 1 else 9000, B, steps=70)
    q = C.area_share_weights(w.surface)
    prob = P.Problem(ctx, torch.from_numpy(w.surface.xyz).cuda(), torch.from_numpy(q).cuda())
    k = P.kernel_struct(w.kernel_kind, *w.kernel)
    f = P.Firing(w.beta, torch.from_numpy(w.theta).cuda())
    a, _, _ = _run(ctx, prob, k, f, w.u0, w.dt, w.steps, False, form=form, B=B)
    g, _, _ = _run(ctx, prob, k, f, w.u0, w.dt, w.steps, True, form=form, B=B)
    assert np.array_equal(a, g)
    nodes, gsteps = _last_graph(ctx)
    assert gsteps == 64 and nodes >= 4 * gsteps
