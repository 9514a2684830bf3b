"""Full-size trajectories against the FP64 oracle's stored end states.

The goldens (tests/golden/make_trajectory_goldens.py, oracle and seeded
workload generators only) hold the oracle's own RBF-QF weights q and u(T) of
the three full-size forward workloads; the GPU runs the same u0, q, kernel,
thresholds, dt and step count through the C ABI:

* torus N = 32768, exponential Mexican hat, one state, dt = 0.02 x 500:
  on-the-fly FP32 (symmetric kernel) and precomputed FP32 W; the whole of u(T);
* ellipsoid N = 65536, 64 states with their own thresholds, dt = 0.05 x 200:
  every form (split W BF16 / FP16, fused on-the-fly split BF16 / FP16, FP32
  vector-unit and FP32 matrix-core sums); u(T) on 4096 seeded rows plus each
  state's largest-|u| row, normalised by each state's max |u(T)| over all rows;
* the 48-problem uneven batch, dt = 0.05 x 100, graph-replayed: every state of
  every problem on up to 512 seeded rows plus its largest-|u| row.

Bounds (relative L-infinity of u(T) per state): 1e-5 for FP32 and the FP16
split forms, 1e-4 for the BF16 split forms (the stated targets).
"""
import os

import numpy as np
import pytest
import torch

from workloads import configs as C

pytestmark = pytest.mark.gpu
P = pytest.importorskip("paper_2504_13379_amd")
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
TOL = {P.FORM_ONTHEFLY_FP32: 1e-5, P.FORM_W_FP32: 1e-5, P.FORM_ONTHEFLY_FP32_MFMA: 1e-5,
       P.FORM_W_FP16X3: 1e-5, P.FORM_ONTHEFLY_FP16X3: 1e-5,
       P.FORM_W_BF16X3: 1e-4, P.FORM_ONTHEFLY_BF16X3: 1e-4}


def _load(name):
    path = os.path.join(GOLDEN, name)
    assert os.path.exists(path), "missing golden %s (run tests/golden/make_trajectory_goldens.py)" % path
    return np.load(path)


def _stream_ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return P.Context(0, torch.cuda.Stream())


def _integrate(ctx, w, q, form, graph=True):
    prob = P.Problem(ctx, torch.from_numpy(w.surface.xyz).cuda(), torch.from_numpy(q).cuda())
    k = P.kernel_struct(w.kernel_kind, *w.kernel)
    th = torch.from_numpy(w.theta).cuda() if w.b > 1 else float(w.theta[0])
    f = P.Firing(w.beta, th)
    W = prob.w_build(k, form) if form in (P.FORM_W_FP32, P.FORM_W_BF16X3, P.FORM_W_FP16X3) else None
    u = torch.from_numpy(w.u0.copy()).cuda()
    prob.integrate(k, f, u, w.dt, w.steps, form=form, W=W, use_graph=graph)
    ctx.stream.synchronize()
    out = u.cpu().numpy()
    del W
    torch.cuda.empty_cache()
    return out


@pytest.mark.parametrize("form", [P.FORM_ONTHEFLY_FP32, P.FORM_W_FP32])
def test_torus_full_trajectory(form):
    g = _load("torus32768_rk4.npz")
    w = C.torus_exp()
    assert w.steps == int(g["steps"]) and w.n == int(g["n"])
    print("trajectory: torus n=%d steps=%d form=%d" % (w.n, w.steps, form), flush=True)
    u = _integrate(_stream_ctx(), w, g["q"], form)
    ref = g["uT"]
    err = np.max(np.abs(u - ref), axis=1) / np.max(np.abs(ref), axis=1)
    print("  rel_linf", err, flush=True)
    assert np.all(err <= TOL[form]), err


@pytest.mark.parametrize("form", [P.FORM_ONTHEFLY_BF16X3, P.FORM_W_BF16X3, P.FORM_ONTHEFLY_FP16X3, P.FORM_W_FP16X3,
                                  P.FORM_ONTHEFLY_FP32_MFMA, P.FORM_ONTHEFLY_FP32])
def test_ellipsoid_ensemble_full_trajectory(form):
    g = _load("ellipsoid65536_rk4.npz")
    w = C.ellipsoid_ensemble()
    assert w.steps == int(g["steps"]) and w.n == int(g["n"])
    print("trajectory: ellipsoid n=%d B=%d steps=%d form=%d" % (w.n, w.b, w.steps, form), flush=True)
    u = _integrate(_stream_ctx(), w, g["q"], form)
    rows = g["rows"]
    err = np.max(np.abs(u[:, rows] - g["uT_rows"]), axis=1) / g["uT_absmax"]
    print("  rel_linf per member: max %.3e median %.3e" % (err.max(), np.median(err)), flush=True)
    assert err.shape == (64,)
    assert np.all(err <= TOL[form]), err


def test_uneven_batch_full_trajectory():
    g = _load("batch48_rk4.npz")
    ws = C.uneven_batch()
    assert len(ws) == len(g["n"]) and ws[0].steps == int(g["steps"])
    ctx = _stream_ctx()
    probs, ks, fs, Bs, states = [], [], [], [], []
    with torch.cuda.stream(ctx.stream):
        for p, w in enumerate(ws):
            assert w.n == int(g["n"][p]) and w.b == int(g["b"][p])
            probs.append(P.Problem(ctx, torch.from_numpy(w.surface.xyz).cuda(),
                                   torch.from_numpy(g["q%02d" % p]).cuda()))
            ks.append(P.kernel_struct(w.kernel_kind, *w.kernel))
            fs.append(P.Firing(w.beta, torch.from_numpy(w.theta).cuda()))
            Bs.append(w.b)
            states.append(torch.from_numpy(w.u0.copy()).cuda())
    torch.cuda.synchronize()
    print("trajectory: uneven batch of %d problems, %d steps" % (len(ws), ws[0].steps), flush=True)
    batch = P.Batch(ctx, probs, ks, fs, Bs)
    batch.integrate(states, ws[0].dt, ws[0].steps, use_graph=True)
    ctx.stream.synchronize()
    worst = 0.0
    for p, (w, u) in enumerate(zip(ws, states)):
        rows = g["rows%02d" % p]
        err = np.max(np.abs(u.cpu().numpy()[:, rows] - g["uT%02d" % p]), axis=1) / g["absmax%02d" % p]
        worst = max(worst, float(err.max()))
        assert np.all(err <= 1e-5), (p, w.name, err)
    print("  worst rel_linf %.3e" % worst, flush=True)
