"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerances come from the arithmetic:
* operator (one application), on-the-fly FP32: every pair term carries a few
  FP32 roundings (coordinates, differences, sqrt/exp, products) plus FP32 sums
  over 256-source tiles, i.e. a relative error of a few 1e-7 of the term;
  compared norm-wise against S_i = sum_j |w_ij q_j f(u_j)|:  |dy_i| <= 1e-5 S_i.
* W_FP32: W and f rounded once to FP32, FP32 row-chunk sums: |dy_i| <= 2e-6 S_i.
* time integration: u(T) to relative L-infinity <= 1e-5 per state (the target
  stated for the FP32 path).
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


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return P.Context(0)


def _abs_scale(x, q, U, kind, p, beta, theta, rows):
    G = q[None, :] * NF.firing(U, beta, theta)
    W = np.abs(NF.kernel_matrix(x, kind, p, rows=rows))
    return np.abs(G) @ W.T


def _run_apply(ctx, x, q, U, kind, p, beta, theta, form):
    prob = P.Problem(ctx, torch.from_numpy(x).cuda(), torch.from_numpy(q).cuda())
    k = P.kernel_struct(kind, *p)
    th = torch.from_numpy(np.asarray(theta, dtype=np.float64)).cuda() if np.ndim(theta) else float(theta)
    f = P.Firing(beta, th)
    u = torch.from_numpy(np.ascontiguousarray(U)).cuda()
    W = prob.w_build(k, form) if form in (P.FORM_W_FP32, P.FORM_W_BF16X3, P.FORM_W_FP16X3) else None
    y = prob.apply(k, f, u, form=form, W=W)
    torch.cuda.synchronize()
    return y.cpu().numpy()


CASES = [(1, 1), (2, 1), (7, 2), (255, 1), (256, 3), (257, 1), (1000, 5), (3001, 2)]


@pytest.mark.parametrize("n,B", CASES)
@pytest.mark.parametrize("kind", [NF.GAUSS_MH, NF.EXP_MH])
@pytest.mark.parametrize("form", [0, 1])
def test_apply_matches_oracle(ctx, n, B, kind, form):
    rng = np.random.default_rng(1000 * n + 10 * B + kind)
    x = S.fibonacci_sphere(n) * rng.uniform(0.9, 1.1)
    q = rng.uniform(0.5, 1.5, size=n) * 4 * math.pi / n
    if n > 3:
        q[rng.integers(n)] *= -0.1
    U = rng.normal(0.2, 0.4, size=(B, n))
    theta = rng.uniform(0.1, 0.3, size=B) if B > 1 else 0.2
    p = GAUSS if kind == NF.GAUSS_MH else EXPK
    y = _run_apply(ctx, x, q, U, kind, p, 20.0, theta, form)
    ref = NF.apply_K(x, q, U, kind, p, 20.0, theta)
    scale = _abs_scale(x, q, U, kind, p, 20.0, theta, None)
    tol = 1e-5 if form == 0 else 2e-6
    err = np.max(np.abs(y - ref) / scale)
    assert err <= tol, err


@pytest.mark.parametrize("form", [0, 6, -1])   # -1: FORM_AUTO
def test_apply_largest_state_count(ctx, form):
    """B = 4096, the largest accepted state count, on a small ragged node set
    (300 nodes): every state against the oracle to 1e-5 of S_i."""
    n, B = 300, 4096
    rng = np.random.default_rng(4096 + form)
    x = S.fibonacci_sphere(n)
    q = rng.uniform(0.5, 1.5, size=n) * 4 * math.pi / n
    U = rng.normal(0.2, 0.4, size=(B, n))
    theta = rng.uniform(0.1, 0.3, size=B)
    y = _run_apply(ctx, x, q, U, NF.GAUSS_MH, GAUSS, 20.0, theta, form)
    ref = NF.apply_K(x, q, U, NF.GAUSS_MH, GAUSS, 20.0, theta)
    scale = _abs_scale(x, q, U, NF.GAUSS_MH, GAUSS, 20.0, theta, None)
    assert np.max(np.abs(y - ref) / scale) <= 1e-5


COINCIDENT_TOL = {0: 1e-5, 1: 2e-6, 4: 4e-5, 5: 1.2e-5, 6: 1e-5}


@pytest.mark.parametrize("form", list(COINCIDENT_TOL))
@pytest.mark.parametrize("kind", [NF.GAUSS_MH, NF.EXP_MH])
def test_apply_coincident_nodes(ctx, form, kind):
    """Nodes that coincide (50 points, each 4 times: r = 0 between distinct
    nodes, not only on the diagonal) in every pair kernel: one state (the
    small-problem path) and 40 states (the matrix-core tiles), against the oracle."""
    rng = np.random.default_rng(50 + form + 7 * kind)
    base = S.fibonacci_sphere(50)
    x = np.repeat(base, 4, axis=0)[rng.permutation(200)]
    n = x.shape[0]
    q = rng.uniform(0.5, 1.5, size=n) * 4 * math.pi / n
    B = 1 if form in (0, 1) else 40
    U = rng.normal(0.2, 0.4, size=(B, n))
    theta = rng.uniform(0.1, 0.3, size=B) if B > 1 else 0.2
    p = GAUSS if kind == NF.GAUSS_MH else EXPK
    y = _run_apply(ctx, x, q, U, kind, p, 20.0, theta, form)
    ref = NF.apply_K(x, q, U, kind, p, 20.0, theta)
    scale = _abs_scale(x, q, U, kind, p, 20.0, theta, None)
    assert np.max(np.abs(y - ref) / scale) <= COINCIDENT_TOL[form]


def test_apply_full_size_torus_sampled_rows(ctx):
    """Torus workload at its full size (N = 32768): one application, 64 sampled rows."""
    w = C.torus_exp()
    x = w.surface.xyz
    q = C.area_share_weights(w.surface)
    rows = np.random.default_rng(5).choice(w.n, 64, replace=False)
    ref = NF.apply_K(x, q, w.u0, w.kernel_kind, w.kernel, w.beta, w.theta, rows=rows)
    scale = _abs_scale(x, q, w.u0, w.kernel_kind, w.kernel, w.beta, w.theta, rows)
    for form in (0, 1):
        y = _run_apply(ctx, x, q, w.u0, w.kernel_kind, w.kernel, w.beta, w.theta, form)
        err = np.max(np.abs(y[:, rows] - ref) / scale)
        assert err <= (1e-5 if form == 0 else 2e-6), (form, err)


def _integrate(ctx, x, q, U, kind, p, beta, theta, dt, steps, form=0, graph=False, ckpt_every=0):
    stream = torch.cuda.Stream() if graph else None
    c = P.Context(0, stream) if graph else ctx
    prob = P.Problem(c, torch.from_numpy(x).cuda(), torch.from_numpy(q).cuda())
    k = P.kernel_struct(kind, *p)
    th = torch.from_numpy(np.asarray(theta, dtype=np.float64)).cuda() if np.ndim(theta) else float(theta)
    f = P.Firing(beta, th)
    u = torch.from_numpy(np.ascontiguousarray(U, dtype=np.float64)).cuda()
    W = prob.w_build(k, form) if form != 0 else None
    ck = prob.integrate(k, f, u, dt, steps, form=form, W=W, use_graph=graph, ckpt_every=ckpt_every)
    torch.cuda.synchronize()
    out = u.cpu().numpy()
    return (out, ck.cpu().numpy()) if ckpt_every else out


@pytest.fixture(scope="module")
def sphere_case():
    w = C.sphere_small()
    q = Q.surface_weights(w.surface)
    op = NF.DenseOperator(w.surface.xyz, q, w.kernel_kind, w.kernel)
    ref = NF.rk4(op, w.u0, w.beta, w.theta, w.dt, w.steps)
    return w, q, ref


def test_integrate_sphere_workload_fp32(ctx, sphere_case):
    """Unit sphere, N = 2000, Gaussian Mexican hat, 50 RK4 steps, FP32 on the fly."""
    w, q, ref = sphere_case
    u = _integrate(ctx, w.surface.xyz, q, w.u0, w.kernel_kind, w.kernel, w.beta, w.theta[0], w.dt, w.steps)
    err = NF.rel_linf(u, ref)
    assert np.all(err <= 1e-5), err


def test_integrate_sphere_workload_w_form(ctx, sphere_case):
    w, q, ref = sphere_case
    u = _integrate(ctx, w.surface.xyz, q, w.u0, w.kernel_kind, w.kernel, w.beta, w.theta[0], w.dt, w.steps, form=1)
    assert np.all(NF.rel_linf(u, ref) <= 1e-5)


@pytest.mark.parametrize("n", [1, 7, 257, 4096, 4097])
@pytest.mark.parametrize("kind", [NF.GAUSS_MH, NF.EXP_MH])
def test_integrate_small_and_ragged(ctx, n, kind):
    """Single-state RK4 at sizes that are mostly padding (1, 7, 257 nodes in
    256-node blocks) and on both sides of the switch from the one-sided
    small-problem path (one launch per stage) to the symmetric one (4096 /
    4097 nodes): 8 steps against the oracle to 1e-5, with a negative weight."""
    rng = np.random.default_rng(70 + n + kind)
    x = S.fibonacci_sphere(n) * rng.uniform(0.9, 1.1)
    q = rng.uniform(0.5, 1.5, size=n) * 4 * math.pi / n
    if n > 3:
        q[rng.integers(n)] *= -0.1
    u0 = rng.normal(0.2, 0.4, size=(1, n))
    p = GAUSS if kind == NF.GAUSS_MH else EXPK
    u = _integrate(ctx, x, q, u0, kind, p, 20.0, 0.2, 0.05, 8)
    ref = NF.rk4(NF.DenseOperator(x, q, kind, p), u0, 20.0, np.array([0.2]), 0.05, 8)
    err = NF.rel_linf(u, ref)
    assert np.all(err <= 1e-5), err


@pytest.fixture(scope="module")
def torus_case():
    w = C.torus_exp(4096, steps=100)
    q = Q.surface_weights(w.surface)
    op = NF.DenseOperator(w.surface.xyz, q, w.kernel_kind, w.kernel)
    return w, q, NF.rk4(op, w.u0, w.beta, w.theta, w.dt, w.steps)


@pytest.mark.parametrize("form", [0, 1])
def test_integrate_torus_exp_kernel(ctx, torus_case, form):
    w, q, ref = torus_case
    u = _integrate(ctx, w.surface.xyz, q, w.u0, w.kernel_kind, w.kernel, w.beta, w.theta[0], w.dt, w.steps, form=form)
    err = NF.rel_linf(u, ref)
    assert np.all(err <= 1e-5), err


def test_integrate_ensemble_per_state_theta(ctx):
    w = C.ellipsoid_ensemble(3000, 5, steps=20)
    q = Q.surface_weights(w.surface)
    op = NF.DenseOperator(w.surface.xyz, q, w.kernel_kind, w.kernel)
    ref = NF.rk4(op, w.u0, w.beta, w.theta, w.dt, w.steps)
    for form in (0, 1):
        u = _integrate(ctx, w.surface.xyz, q, w.u0, w.kernel_kind, w.kernel, w.beta, w.theta, w.dt, w.steps, form)
        err = NF.rel_linf(u, ref)
        assert np.all(err <= 1e-5), (form, err)


def test_integrate_beta_zero_closed_form_full_size(ctx):
    """beta = 0: u_n = b + R(-dt)^n (u0 - b), b_i = K_i = sum_j w_ij q_j / 2 (f = 1/2),
    checked at sampled rows of the full-size torus workload (N = 32768)."""
    w = C.torus_exp()
    x = w.surface.xyz
    q = C.area_share_weights(w.surface)
    steps = 20
    u = _integrate(ctx, x, q, w.u0, w.kernel_kind, w.kernel, 0.0, 0.25, w.dt, steps)
    rows = np.random.default_rng(6).choice(w.n, 64, replace=False)
    b = NF.apply_K(x, q, np.zeros((1, w.n)), w.kernel_kind, w.kernel, 0.0, 0.25, rows=rows)[0]
    z = -w.dt
    R = (1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24) ** steps
    expect = b + R * (w.u0[0, rows] - b)
    assert np.max(np.abs(u[0, rows] - expect)) <= 1e-5 * np.max(np.abs(expect))


def test_integrate_deterministic_graph_and_resume(ctx, sphere_case):
    w, q, _ = sphere_case
    args = (w.surface.xyz, q, w.u0, w.kernel_kind, w.kernel, w.beta, w.theta[0], w.dt)
    a = _integrate(ctx, *args, 30)
    b = _integrate(ctx, *args, 30)
    g = _integrate(ctx, *args, 30, graph=True)
    assert np.array_equal(a, b)
    assert np.array_equal(a, g)
    half = _integrate(ctx, *args, 15)
    resumed = _integrate(ctx, w.surface.xyz, q, half, w.kernel_kind, w.kernel, w.beta, w.theta[0], w.dt, 15)
    assert np.array_equal(a, resumed)
    full, ck = _integrate(ctx, *args, 30, ckpt_every=10)
    assert ck.shape == (4, 1, w.n)
    assert np.array_equal(ck[0], w.u0)
    assert np.array_equal(ck[3], a)
    assert np.array_equal(ck[1], _integrate(ctx, *args, 10))


@pytest.mark.parametrize("n", [1000, 2000, 5000])
def test_integrate_ignores_stale_workspace(ctx, n):
    """A workspace may hold anything before a call (here 0xFF bytes, NaN
    patterns): RK4 and Adams-Bashforth 5 runs give bitwise the results of a
    zeroed workspace, and RK4 stays within 1e-5 of the oracle.  Sizes on both
    sides of the switch between the one-sided small-problem path (one launch
    per stage, sources alternating between two buffers) and the symmetric one."""
    w = C.sphere_small(n)
    q = C.area_share_weights(w.surface)
    prob = P.Problem(ctx, torch.from_numpy(w.surface.xyz).cuda(), torch.from_numpy(q).cuda())
    k = P.kernel_struct(w.kernel_kind, *w.kernel)
    f = P.Firing(w.beta, float(w.theta[0]))
    lib = P.lib()
    out = {}
    for fill in (0, 255):
        ws = torch.full((lib.nfr_integrate_ab5_workspace_size(prob.handle, 1, 0),), fill, dtype=torch.uint8,
                        device="cuda")
        u = torch.from_numpy(w.u0.copy()).cuda()
        prob.integrate(k, f, u, 0.05, 12, ws=ws)
        ws.fill_(fill)
        v = torch.from_numpy(w.u0.copy()).cuda()
        prob.integrate_ab5(k, f, v, 0.05, 9, ws=ws)
        torch.cuda.synchronize()
        out[fill] = (u.cpu().numpy(), v.cpu().numpy())
    assert np.array_equal(out[0][0], out[255][0]) and np.array_equal(out[0][1], out[255][1])
    ref = NF.rk4(NF.DenseOperator(w.surface.xyz, q, w.kernel_kind, w.kernel), w.u0, w.beta, w.theta, 0.05, 12)
    assert np.all(NF.rel_linf(out[0][0], ref) <= 1e-5)


def test_invalid_arguments_rejected(ctx):
    x = S.fibonacci_sphere(100)
    prob = P.Problem(ctx, torch.from_numpy(x).cuda(), torch.full((100,), 0.1, dtype=torch.float64).cuda())
    u = torch.zeros((1, 100), dtype=torch.float64, device="cuda")
    f = P.Firing(20.0, 0.2)
    with pytest.raises(P.NfrError) as e:
        prob.apply(P.kernel_struct(0, 1.0, -0.15, 0.5, 0.4), f, u)
    assert e.value.status == -1
    with pytest.raises(P.NfrError) as e:
        prob.apply(P.kernel_struct(0, float("nan"), 0.15, 0.5, 0.4), f, u)
    assert e.value.status == -2
    with pytest.raises(P.NfrError):
        prob.integrate(P.kernel_struct(0, *GAUSS), f, u, -0.1, 3)
    with pytest.raises(P.NfrError):
        prob.apply(P.kernel_struct(0, *GAUSS), f, u, form=1, W=None)
    with pytest.raises(P.NfrError) as e:
        prob.apply(P.kernel_struct(7, *GAUSS), f, u)
    assert e.value.status == -1


# Length scales in an integer ratio: the symmetric kernel takes exp2(-t) as a
# power of exp2(-rho t) (rho = 1/m); same tolerance as the two-exponential form.
RATIO_KERNELS = [(NF.GAUSS_MH, (1.0, 0.2, 0.5, 0.2 * math.sqrt(2.0))),     # rho = 1/2
                 (NF.GAUSS_MH, (1.0, 0.12, 0.4, 0.12 * math.sqrt(3.0))),   # rho = 1/3
                 (NF.EXP_MH, (1.0, 0.1, 0.5, 0.2)),                        # rho = 1/2
                 (NF.EXP_MH, (2.0, 0.1, 1.0, 0.4)),                        # rho = 1/4
                 (NF.GAUSS_MH, (1.0, 0.1, 0.3, 0.2))]                      # rho = 1/4


@pytest.mark.parametrize("kind,p", RATIO_KERNELS)
@pytest.mark.parametrize("n", [383, 3001, 5000, 9000])   # one-sided small; symmetric 64- and 256-node tiles
def test_apply_integer_ratio_kernels(ctx, kind, p, n):
    rng = np.random.default_rng(n + int(p[3] * 1000))
    x = S.fibonacci_sphere(n)
    q = rng.uniform(0.5, 1.5, size=n) * 4 * math.pi / n
    U = rng.normal(0.2, 0.4, size=(1, n))
    y = _run_apply(ctx, x, q, U, kind, p, 20.0, 0.2, 0)
    ref = NF.apply_K(x, q, U, kind, p, 20.0, 0.2)
    scale = _abs_scale(x, q, U, kind, p, 20.0, 0.2, None)
    assert np.max(np.abs(y - ref) / scale) <= 1e-5


@pytest.mark.parametrize("kind,p", RATIO_KERNELS)
def test_integrate_integer_ratio_kernels_small(ctx, kind, p):
    """The one-launch RK4 stage of small single-state problems for every
    integer-ratio kernel: 6 steps against the oracle to 1e-5."""
    n = 383
    rng = np.random.default_rng(7 + int(p[3] * 1000))
    x = S.fibonacci_sphere(n)
    q = rng.uniform(0.5, 1.5, size=n) * 4 * math.pi / n
    u0 = rng.normal(0.2, 0.4, size=(1, n))
    u = _integrate(ctx, x, q, u0, kind, p, 20.0, 0.2, 0.05, 6)
    ref = NF.rk4(NF.DenseOperator(x, q, kind, p), u0, 20.0, np.array([0.2]), 0.05, 6)
    assert np.all(NF.rel_linf(u, ref) <= 1e-5)


@pytest.mark.parametrize("n", [300000, 700000])
def test_apply_large_n_both_sides_of_the_slot_budget(ctx, n):
    """Single-state on-the-fly sums at N = 3e5 (symmetric kernel, 2.8 GB of tile slots)
    and N = 7e5 (beyond the 8 GiB slot budget: the one-sided kernel), sampled rows."""
    rng = np.random.default_rng(n)
    x = S.fibonacci_sphere(n)
    q = np.full(n, 4 * math.pi / n) * rng.uniform(0.9, 1.1, size=n)
    U = rng.normal(0.2, 0.4, size=(1, n))
    y = _run_apply(ctx, x, q, U, NF.EXP_MH, EXPK, 20.0, 0.2, 0)
    rows = rng.choice(n, 24, replace=False)
    ref = NF.apply_K(x, q, U, NF.EXP_MH, EXPK, 20.0, 0.2, rows=rows)
    scale = _abs_scale(x, q, U, NF.EXP_MH, EXPK, 20.0, 0.2, rows)
    assert np.max(np.abs(y[:, rows] - ref) / scale) <= 1e-5


# The forward pair sums accumulate w / A_e (u = e1 - (A_i / A_e) e2); a kernel
# without an excitatory part is rewritten as its single inhibitory term.
# Amplitude edge cases for every form, with one negative weight; tolerances
# as above (split forms: those derived in test_gpu_mfma_otf / test_gpu_mfma).
AMP_CASES = [(0.0, 0.5), (-1.0, 0.5), (1e-6, 0.5), (0.7, 0.0), (0.0, 0.0)]
FORM_TOL = {(0, 1): 1e-5, (0, 5): 1e-5, (1, 5): 2e-6, (2, 40): 3e-5, (3, 40): 2e-6, (4, 40): 4e-5, (5, 40): 1.2e-5,
            (6, 40): 1e-5}


@pytest.mark.parametrize("form,B", list(FORM_TOL))
@pytest.mark.parametrize("Ae,Ai", AMP_CASES)
@pytest.mark.parametrize("kind", [NF.GAUSS_MH, NF.EXP_MH])
def test_apply_amplitude_edge_cases(ctx, form, B, Ae, Ai, kind):
    n = 1100
    rng = np.random.default_rng(17 + B + 3 * form + kind)
    x = S.fibonacci_sphere(n)
    q = rng.uniform(0.5, 1.5, size=n) * 4 * math.pi / n
    q[rng.integers(n)] *= -0.2
    U = rng.normal(0.2, 0.4, size=(B, n))
    theta = rng.uniform(0.1, 0.3, size=B) if B > 1 else 0.2
    p = (Ae, 0.15, Ai, 0.45) if kind == NF.GAUSS_MH else (Ae, 0.1, Ai, 0.3)   # the exponential one: ratio 1/3
    y = _run_apply(ctx, x, q, U, kind, p, 20.0, theta, form)
    ref = NF.apply_K(x, q, U, kind, p, 20.0, theta)
    if Ae == 0.0 and Ai == 0.0:
        assert np.all(y == 0.0)
        return
    scale = _abs_scale(x, q, U, kind, p, 20.0, theta, None)
    err = np.max(np.abs(y - ref) / scale)
    assert err <= FORM_TOL[(form, B)], err
