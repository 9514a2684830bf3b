"""GPU parity of the uneven batch (one persistent pair-sum launch per stage for
all problems) against the FP64 oracle, problem by problem and state by state.
Tolerance: u(T) to relative L-infinity 1e-5 per state (FP32 pair sums)."""
import numpy as np
import pytest
import torch

from oracle import neural_field as NF
from oracle import quadrature as Q
from workloads import configs as C
from workloads import surfaces as S

pytestmark = pytest.mark.gpu
P = pytest.importorskip("paper_2504_13379_amd")


@pytest.fixture(scope="module")
def gctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    stream = torch.cuda.Stream()
    return P.Context(0, stream)


def _mixed_batch(seed=5):
    rng = np.random.default_rng(seed)
    specs = [("sphere", 300, 1, 0), ("torus", 900, 4, 1), ("ellipsoid", 1500, 16, 0), ("bumpy", 500, 1, 0),
             ("sphere", 2100, 4, 1), ("torus", 1300, 1, 0), ("ellipsoid", 257, 3, 1)]
    out = []
    for kind, n, B, kk in specs:
        surf = S.make_surface(kind, n, rng)
        q = Q.surface_weights(surf) if n >= 1000 else C.area_share_weights(surf) * rng.uniform(0.9, 1.1, size=n)
        kern = (1.0, 0.15, 0.5, 0.4) if kk == 0 else (2.0, 0.1, 1.0, 0.3)
        kern = tuple(v * rng.uniform(0.9, 1.1) for v in kern)
        theta = rng.uniform(0.15, 0.3, size=B)
        u0 = np.stack([C.bump(surf.xyz, surf.xyz[rng.integers(n)]) for _ in range(B)])
        out.append((surf, q, kk, kern, 20.0, theta, u0))
    return out


def _make(gctx, specs):
    probs, ks, fs, Bs, states = [], [], [], [], []
    with torch.cuda.stream(gctx.stream):
        for surf, q, kk, kern, beta, theta, u0 in specs:
            probs.append(P.Problem(gctx, torch.from_numpy(surf.xyz).cuda(), torch.from_numpy(q).cuda()))
            ks.append(P.kernel_struct(kk, *kern))
            fs.append(P.Firing(beta, torch.from_numpy(theta).cuda()))
            Bs.append(u0.shape[0])
            states.append(torch.from_numpy(u0.copy()).cuda())
    torch.cuda.synchronize()
    return P.Batch(gctx, probs, ks, fs, Bs), states, probs


def test_batch_matches_oracle_per_problem_and_graph_is_bitwise(gctx):
    specs = _mixed_batch()
    dt, steps = 0.05, 12
    batch, states, _ = _make(gctx, specs)
    batch.integrate(states, dt, steps, use_graph=False)
    torch.cuda.synchronize()
    eager = [s.cpu().numpy() for s in states]
    batch2, states2, _ = _make(gctx, specs)
    batch2.integrate(states2, dt, steps, use_graph=True)
    torch.cuda.synchronize()
    for a, s in zip(eager, states2):
        assert np.array_equal(a, s.cpu().numpy())
    for (surf, q, kk, kern, beta, theta, u0), u in zip(specs, eager):
        ref = NF.rk4(NF.DenseOperator(surf.xyz, q, kk, kern), u0, beta, theta, dt, steps)
        err = NF.rel_linf(u, ref)
        assert np.all(err <= 1e-5), (surf.kind, surf.n, err)


def test_batch_tuned_configuration_keeps_parity(gctx):
    specs = _mixed_batch(seed=9)[:4]
    dt, steps = 0.05, 6
    batch, states, _ = _make(gctx, specs)
    best = batch.tune(states)
    chunk, wgs = batch.config
    assert best > 0 and chunk % 256 == 0 and wgs >= 1
    batch.integrate(states, dt, steps, use_graph=True)
    torch.cuda.synchronize()
    for (surf, q, kk, kern, beta, theta, u0), u in zip(specs, states):
        ref = NF.rk4(NF.DenseOperator(surf.xyz, q, kk, kern), u0, beta, theta, dt, steps)
        assert np.all(NF.rel_linf(u.cpu().numpy(), ref) <= 1e-5)


def test_batch_full_size_uneven_workload_beta_zero(gctx):
    """The 48-problem uneven batch at full size (N up to 40000, B in {1, 4, 16}) with beta = 0:
    u_n = b + R(-dt)^n (u0 - b), b_i = K_i, checked at sampled rows of every problem."""
    ws = C.uneven_batch(steps=4)
    specs = []
    for w in ws:
        q = C.area_share_weights(w.surface)
        specs.append((w.surface, q, w.kernel_kind, w.kernel, 0.0, w.theta, w.u0))
    batch, states, _ = _make(gctx, specs)
    batch.integrate(states, 0.05, 4, use_graph=True)
    torch.cuda.synchronize()
    z = -0.05
    R = (1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24) ** 4
    rng = np.random.default_rng(0)
    for (surf, q, kk, kern, beta, theta, u0), u in zip(specs, states):
        rows = rng.choice(surf.n, 8, replace=False)
        b = NF.apply_K(surf.xyz, q, np.zeros((1, surf.n)), kk, kern, 0.0, 0.2, rows=rows)[0]
        expect = b[None, :] + R * (u0[:, rows] - b[None, :])
        got = u.cpu().numpy()[:, rows]
        assert np.max(np.abs(got - expect)) <= 1e-5 * np.max(np.abs(expect)), (surf.kind, surf.n)


def test_batch_amplitude_edge_cases(gctx):
    """Problems whose kernels have no excitatory part, a negative one, or vanish entirely
    (the pair sums accumulate w / A_e, such kernels are rewritten first)."""
    rng = np.random.default_rng(9)
    specs = []
    for kind, n, B, kern in (("sphere", 700, 4, (0.0, 0.15, 0.5, 0.4)), ("torus", 900, 1, (-1.0, 0.15, 0.5, 0.4)),
                             ("ellipsoid", 600, 16, (0.0, 0.15, 0.0, 0.4)), ("sphere", 500, 3, (1.0, 0.15, 0.5, 0.4))):
        surf = S.make_surface(kind, n, rng)
        q = C.area_share_weights(surf) * rng.uniform(0.9, 1.1, size=n)
        theta = rng.uniform(0.15, 0.3, size=B)
        u0 = np.stack([C.bump(surf.xyz, surf.xyz[rng.integers(n)]) for _ in range(B)])
        specs.append((surf, q, 0, kern, 20.0, theta, u0))
    dt, steps = 0.05, 8
    batch, states, _ = _make(gctx, specs)
    batch.integrate(states, dt, steps, use_graph=True)
    torch.cuda.synchronize()
    for (surf, q, kk, kern, beta, theta, u0), u in zip(specs, states):
        ref = NF.rk4(NF.DenseOperator(surf.xyz, q, kk, kern), u0, beta, theta, dt, steps)
        err = NF.rel_linf(u.cpu().numpy(), ref)
        assert np.all(err <= 1e-5), (surf.kind, kern, err)
