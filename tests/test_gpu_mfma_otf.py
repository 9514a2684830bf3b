"""GPU parity of the fused on-the-fly split forms (ONTHEFLY_BF16X3 = 4,
ONTHEFLY_FP16X3 = 5): W evaluated in FP32 by the vector units, split into
hi + 2^-c lo in registers and multiplied on the matrix cores.

Tolerances add the two error sources already bounded for the other forms
(norm-wise against S_i = sum_j |w_ij q_j f(u_j)|):
* the FP32 evaluation of each W entry, as in the on-the-fly FP32 form
  (coordinate, difference, exp2 roundings; also the scaled period):
  |dy_i| <= 1e-5 S_i; the BF16 form evaluates Gaussian kernels on
  non-periodic surfaces by the norm expansion of r^2 while sig^2 max|x|^2
  <= 96 (for the steeper exponential), whose roundings keep each entry within
  3e-5 of itself;
* the hi/lo split of W and f(u) with FP32 accumulation, as in the W_* split
  forms: 3e-5 S_i (BF16), 2e-6 S_i (FP16).
Hence 6e-5 (BF16) and 1.2e-5 (FP16) for one application; trajectories
u(T): 1e-4 (BF16, the split-BF16 target) and 2e-5 (FP16: the FP32 path's
1e-5 plus the split form's 1e-5) relative L-infinity per state.
FP16 also has an absolute floor: a lifted source value q_j f 2^sG (sG = 14 -
ceil(log2 max q)) below FP16's normal range keeps its hi part and its
remainder (lifted by 2^11) on the subnormal grid of spacing 2^-24, so it is
represented to 2^-36 in lifted units; one application is then within
1.2e-5 S_i + 2^-36 2^-sG sum_j |w_ij|.  The floor matters only where S_i is
made of such quiet sources alone (a single node, B = 40, below).
"""
import ctypes
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
TOL_APPLY = {4: 6e-5, 5: 1.2e-5}
TOL_STATE = {4: 1e-4, 5: 2e-5}
L = 2.0 * math.pi


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return P.Context(0)


def _apply(ctx, x, q, U, kind, p, beta, theta, form, period=0.0):
    prob = P.Problem(ctx, torch.from_numpy(x).cuda(), torch.from_numpy(q).cuda(), period=period)
    k = P.kernel_struct(kind, *p)
    th = torch.from_numpy(np.asarray(theta, dtype=np.float64)).cuda() if np.ndim(theta) else float(theta)
    y = prob.apply(k, P.Firing(beta, th), torch.from_numpy(np.ascontiguousarray(U)).cuda(), form=form)
    torch.cuda.synchronize()
    return y.cpu().numpy()


def _scale(x, q, U, kind, p, beta, theta, rows=None, period=None):
    G = q[None, :] * NF.firing(U, beta, theta)
    return np.abs(G) @ np.abs(NF.kernel_matrix(x, kind, p, rows=rows, period=period)).T


@pytest.mark.parametrize("form", [4, 5])
@pytest.mark.parametrize("n,B", [(1, 1), (1, 40), (200, 3), (256, 32), (257, 64), (300, 33), (1000, 64), (2500, 70),
                                 (1100, 130)])
@pytest.mark.parametrize("kind", [NF.GAUSS_MH, NF.EXP_MH])
def test_fused_apply_matches_oracle(ctx, form, n, B, kind):
    rng = np.random.default_rng(7 * n + B + 100 * form + kind)
    x = S.fibonacci_sphere(n) * 1.05
    q = rng.uniform(0.5, 1.5, size=n) * 4 * math.pi / n
    U = rng.normal(0.2, 0.4, size=(B, n))
    theta = rng.uniform(0.15, 0.3, size=B)
    p = GAUSS if kind == NF.GAUSS_MH else EXPK
    y = _apply(ctx, x, q, U, kind, p, 20.0, theta, form)
    ref = NF.apply_K(x, q, U, kind, p, 20.0, theta)
    scale = _scale(x, q, U, kind, p, 20.0, theta)
    floor = _fp16_floor(x, q, kind, p) if form == 5 else 0.0
    err = np.max(np.abs(y - ref) / scale)
    print("fused form %d, kind %d, n = %d, B = %d: max |dy| / S = %.3e" % (form, kind, n, B, err), flush=True)
    assert np.all(np.abs(y - ref) <= TOL_APPLY[form] * scale + floor), err


def _fp16_floor(x, q, kind, p):
    """2^-36 2^-sG sum_j |w_ij| per target (see the module docstring)."""
    f, e = math.frexp(float(np.max(np.abs(q))))
    sG = 14 - (e - 1 if f == 0.5 else e)
    return 2.0 ** (-36 - sG) * np.abs(NF.kernel_matrix(x, kind, p)).sum(axis=1)[None, :]


@pytest.mark.parametrize("form", [4, 5])
def test_fused_largest_state_count(ctx, form):
    """B = 4096, the largest accepted state count (64 groups of 64 states; for
    BF16 the eight-wave far form in tile order), on a ragged node set of 300
    nodes: every state against the oracle to the form's bound."""
    n, B = 300, 4096
    rng = np.random.default_rng(4096 + 17 * form)
    x = S.fibonacci_sphere(n)
    q = rng.uniform(0.5, 1.5, size=n) * 4 * math.pi / n
    U = rng.normal(0.2, 0.4, size=(B, n))
    theta = rng.uniform(0.1, 0.3, size=B)
    y = _apply(ctx, x, q, U, NF.GAUSS_MH, GAUSS, 20.0, theta, form)
    ref = NF.apply_K(x, q, U, NF.GAUSS_MH, GAUSS, 20.0, theta)
    err = np.max(np.abs(y - ref) / _scale(x, q, U, NF.GAUSS_MH, GAUSS, 20.0, theta))
    print("fused form %d, n = %d, B = %d: max |dy| / S = %.3e" % (form, n, B, err), flush=True)
    assert err <= TOL_APPLY[form], err


# Integer length ratios rho = 1/m: the excitatory exponential is taken as a
# power of the inhibitory one, coordinates scaled by the inhibitory length.
RATIO_KERNELS = [(NF.GAUSS_MH, (1.0, 0.2, 0.5, 0.2 * math.sqrt(2.0))),     # rho = 1/2
                 (NF.GAUSS_MH, (1.0, 0.12, 0.4, 0.12 * math.sqrt(3.0))),   # rho = 1/3
                 (NF.EXP_MH, (2.0, 0.1, 1.0, 0.4)),                        # rho = 1/4
                 (NF.GAUSS_MH, (1.0, 0.1, 0.3, 0.2))]                      # rho = 1/4


@pytest.mark.parametrize("form", [4, 5])
@pytest.mark.parametrize("kind,p", RATIO_KERNELS)
def test_fused_integer_ratio_kernels(ctx, form, kind, p):
    n, B = 1500, 40
    rng = np.random.default_rng(n + int(p[3] * 1000) + form)
    x = S.fibonacci_sphere(n)
    q = rng.uniform(0.5, 1.5, size=n) * 4 * math.pi / n
    U = rng.normal(0.2, 0.4, size=(B, n))
    y = _apply(ctx, x, q, U, kind, p, 20.0, 0.2, form)
    ref = NF.apply_K(x, q, U, kind, p, 20.0, 0.2)
    assert np.max(np.abs(y - ref) / _scale(x, q, U, kind, p, 20.0, 0.2)) <= TOL_APPLY[form]


@pytest.mark.parametrize("form", [4, 5])
@pytest.mark.parametrize("kind,p", [(NF.GAUSS_MH, (1.0, 0.6, 0.5, 1.2)), (NF.EXP_MH, (2.0, 0.5, 1.0, 1.5)),
                                    (NF.GAUSS_MH, (1.0, 0.5, 0.5, 1.0))])   # the last: rho = 1/4
def test_fused_periodic_plane(ctx, form, kind, p):
    """Doubly periodic square of side 2 pi (eq. dist), 8 states."""
    rng = np.random.default_rng(40 + form + kind)
    surf = S.flat_square(2000, L, rng, 0.3)
    q = Q.plane_weights(surf.xyz)
    B = 8
    U = rng.normal(0.3, 0.4, size=(B, surf.n))
    theta = rng.uniform(0.1, 0.4, size=B)
    y = _apply(ctx, surf.xyz, q, U, kind, p, 5.0, theta, form, period=L)
    ref = NF.apply_K(surf.xyz, q, U, kind, p, 5.0, theta, period=L)
    err = np.max(np.abs(y - ref) / _scale(surf.xyz, q, U, kind, p, 5.0, theta, period=L))
    assert err <= TOL_APPLY[form], err


def test_fused_fp16_scaling_handles_tiny_weights(ctx):
    """Weights ~1e-7 would underflow FP16 without the power-of-two lift of W."""
    n, B = 700, 8
    rng = np.random.default_rng(3)
    x = S.fibonacci_sphere(n)
    q = rng.uniform(0.5, 1.5, size=n) * 1e-7
    U = rng.normal(0.2, 0.4, size=(B, n))
    y = _apply(ctx, x, q, U, NF.GAUSS_MH, GAUSS, 20.0, 0.2, 5)
    ref = NF.apply_K(x, q, U, NF.GAUSS_MH, GAUSS, 20.0, 0.2)
    assert np.max(np.abs(y - ref) / _scale(x, q, U, NF.GAUSS_MH, GAUSS, 20.0, 0.2)) <= TOL_APPLY[5]


def test_fused_matches_w_form_of_same_precision(ctx):
    """Same products as the BF16 W form; they differ only by the FP32 (fused,
    norm expansion) against FP64 (W build) evaluation of W before the split."""
    n, B = 2000, 64
    rng = np.random.default_rng(5)
    x = S.fibonacci_sphere(n)
    q = rng.uniform(0.5, 1.5, size=n) * 4 * math.pi / n
    U = rng.normal(0.2, 0.4, size=(B, n))
    theta = rng.uniform(0.15, 0.3, size=B)
    prob = P.Problem(ctx, torch.from_numpy(x).cuda(), torch.from_numpy(q).cuda())
    k = P.kernel_struct(NF.GAUSS_MH, *GAUSS)
    f = P.Firing(20.0, torch.from_numpy(theta).cuda())
    u = torch.from_numpy(U).cuda()
    yw = prob.apply(k, f, u, form=2, W=prob.w_build(k, 2)).cpu().numpy()
    yf = prob.apply(k, f, u, form=4).cpu().numpy()
    yf2 = prob.apply(k, f, u, form=4).cpu().numpy()
    assert np.array_equal(yf, yf2)
    scale = _scale(x, q, U, NF.GAUSS_MH, GAUSS, 20.0, theta)
    assert np.max(np.abs(yf - yw) / scale) <= 3e-5 + 2 * 3e-5


@pytest.mark.parametrize("shift", [0.0, 0.45, 3.0])
def test_fused_bf16_translation_invariance_across_r2_paths(ctx, shift):
    """The operator is invariant under translation.  On the unit sphere with the
    ensemble's Gaussian (sig^2 = log2(e) / 0.15^2 = 64.1) the shifts put
    sig^2 max|x|^2 at 64 (norm expansion), 135 and 1026 (differences): each
    result matches the oracle on the unshifted sphere."""
    n, B = 1500, 40
    rng = np.random.default_rng(77)
    x = S.fibonacci_sphere(n)
    q = rng.uniform(0.5, 1.5, size=n) * 4 * math.pi / n
    U = rng.normal(0.2, 0.4, size=(B, n))
    theta = rng.uniform(0.15, 0.3, size=B)
    xs = x + np.array([shift, 0.0, 0.0])
    y = _apply(ctx, xs, q, U, NF.GAUSS_MH, GAUSS, 20.0, theta, 4)
    ref = NF.apply_K(x, q, U, NF.GAUSS_MH, GAUSS, 20.0, theta)
    err = np.max(np.abs(y - ref) / _scale(x, q, U, NF.GAUSS_MH, GAUSS, 20.0, theta))
    print("fused form 4, unit sphere shifted by %.2f: max |dy| / S = %.3e" % (shift, err), flush=True)
    assert err <= TOL_APPLY[4], err


@pytest.mark.parametrize("form", [4, 5])
def test_fused_full_size_ellipsoid_sampled_rows(ctx, form):
    """Ellipsoid ensemble at its full size (N = 65536, B = 64): one application, sampled rows."""
    w = C.ellipsoid_ensemble()
    x = w.surface.xyz
    q = C.area_share_weights(w.surface)
    rows = np.random.default_rng(12).choice(w.n, 24, replace=False)
    y = _apply(ctx, x, q, w.u0, w.kernel_kind, w.kernel, w.beta, w.theta, form)
    ref = NF.apply_K(x, q, w.u0, w.kernel_kind, w.kernel, w.beta, w.theta, rows=rows)
    err = np.max(np.abs(y[:, rows] - ref) / _scale(x, q, w.u0, w.kernel_kind, w.kernel, w.beta, w.theta, rows))
    print("fused form %d, N = %d, B = %d: one application, max |dy| / S over 24 rows = %.3e" % (form, w.n, w.b, err),
          flush=True)
    assert err <= TOL_APPLY[form], err


@pytest.fixture(scope="module")
def ensemble_case():
    w = C.ellipsoid_ensemble(3000, 64, steps=30)
    q = Q.surface_weights(w.surface)
    op = NF.DenseOperator(w.surface.xyz, q, w.kernel_kind, w.kernel)
    return w, q, NF.rk4(op, w.u0, w.beta, w.theta, w.dt, w.steps)


@pytest.mark.parametrize("form", [4, 5])
@pytest.mark.parametrize("use_graph", [False, True])
def test_fused_integrate_ensemble_per_member(ctx, ensemble_case, form, use_graph):
    w, q, ref = ensemble_case
    c = P.Context(0, torch.cuda.Stream()) if use_graph else ctx
    prob = P.Problem(c, torch.from_numpy(w.surface.xyz).cuda(), torch.from_numpy(q).cuda())
    k = P.kernel_struct(w.kernel_kind, *w.kernel)
    u = torch.from_numpy(w.u0.copy()).cuda()
    prob.integrate(k, P.Firing(w.beta, torch.from_numpy(w.theta).cuda()), u, w.dt, w.steps, form=form,
                   use_graph=use_graph)
    torch.cuda.synchronize()
    err = NF.rel_linf(u.cpu().numpy(), ref)
    print("fused form %d, ensemble N = %d, %d steps, graph %s: max member error %.3e" % (form, w.n, w.steps, use_graph,
                                                                                       err.max()), flush=True)
    assert err.shape == (64,)
    assert np.all(err <= TOL_STATE[form]), err.max()


def test_fused_form_needs_no_w(ctx):
    assert P.lib().nfr_w_bytes(1000, 4) == 0 and P.lib().nfr_w_bytes(1000, 5) == 0
    x = S.fibonacci_sphere(300)
    prob = P.Problem(ctx, torch.from_numpy(x).cuda(), torch.full((300,), 4 * math.pi / 300, dtype=torch.float64).cuda())
    with pytest.raises(ValueError):
        prob.w_build(P.kernel_struct(0, *GAUSS), 4)
    k = P.kernel_struct(0, *GAUSS)
    for form in (4, 5):   # rejected before the (NULL) buffer is looked at
        assert P.lib().nfr_w_build(prob.handle, ctypes.byref(k), form, None, 0) == -1


@pytest.mark.parametrize("form", [4, 5])
def test_fused_large_n_sampled_rows(ctx, form):
    """N = 262144, B = 64 (the split-W form would need 275 GB of W here): one application,
    24 sampled rows against the oracle."""
    n, B = 262144, 64
    rng = np.random.default_rng(21 + form)
    x = S.fibonacci_sphere(n) * 1.05
    q = np.full(n, 4 * math.pi * 1.05 ** 2 / n) * rng.uniform(0.9, 1.1, size=n)
    U = rng.normal(0.2, 0.4, size=(B, n))
    theta = rng.uniform(0.15, 0.3, size=B)
    y = _apply(ctx, x, q, U, NF.GAUSS_MH, GAUSS, 20.0, theta, form)
    rows = rng.choice(n, 24, replace=False)
    ref = NF.apply_K(x, q, U, NF.GAUSS_MH, GAUSS, 20.0, theta, rows=rows)
    err = np.max(np.abs(y[:, rows] - ref) / _scale(x, q, U, NF.GAUSS_MH, GAUSS, 20.0, theta, rows))
    print("fused form %d, N = %d, B = %d: max |dy| / S over 24 rows = %.3e" % (form, n, B, err), flush=True)
    assert err <= TOL_APPLY[form], err


# ---------------------------------------------------------------- tile order and far blocks

def _two_caps(n, gap):
    """n nodes on two copies of a cap of the unit sphere (chordal radius about
    0.35), moved so that their centres sit at x = -gap/2 and x = gap/2."""
    x = S.fibonacci_sphere(40 * n)
    a = x[x[:, 2] > 0.94][: n // 2] - np.array([0.0, 0.0, 0.97])
    assert a.shape[0] == n // 2
    return np.concatenate([a - np.array([gap / 2, 0.0, 0.0]), a + np.array([gap / 2, 0.0, 0.0])])


def test_far_blocks_eligibility(ctx):
    """nfr_far_blocks: some but not all blocks of the ellipsoid ensemble's kernel are far;
    kernels outside the far path's conditions report none."""
    w = C.ellipsoid_ensemble(4000, 8, steps=1)
    q = C.area_share_weights(w.surface)
    prob = P.Problem(ctx, torch.from_numpy(w.surface.xyz).cuda(), torch.from_numpy(q).cuda())
    far, tot = prob.far_blocks(P.kernel_struct(NF.GAUSS_MH, *GAUSS))
    npad = prob.npad
    assert tot == (npad // 32) * (npad // 16)
    assert 0.2 * tot < far < tot, (far, tot)
    for kind, p in [(NF.EXP_MH, EXPK),                             # exponential kernel
                    (NF.GAUSS_MH, (1.0, 0.15, 0.0, 0.4)),          # no inhibitory term
                    (NF.GAUSS_MH, (1.0, 0.36, 0.5, 0.4)),          # rho = 0.81 > 3/4
                    (NF.GAUSS_MH, (1.0, 0.2, 0.5, 0.2 * math.sqrt(2.0)))]:   # integer ratio (one exponential)
        assert prob.far_blocks(P.kernel_struct(kind, *p))[0] == 0, (kind, p)
    rng = np.random.default_rng(8)
    flat = S.flat_square(2000, L, rng, 0.3)
    per = P.Problem(ctx, torch.from_numpy(flat.xyz).cuda(), torch.from_numpy(Q.plane_weights(flat.xyz)).cuda(),
                    period=L)
    assert per.far_blocks(P.kernel_struct(NF.GAUSS_MH, 1.0, 0.3, 0.5, 0.8))[0] == 0   # periodic


@pytest.mark.parametrize("gap", [1.2, 1.6])
def test_fused_far_blocks_two_caps(ctx, gap):
    """Two caps `gap` apart (1.2: the caps' nearest nodes 0.5 apart, so some blocks
    between them are near; 1.6: every block between them is far), the blocks
    within a cap near: far blocks evaluate only the inhibitory exponential, and
    one application matches the oracle, which evaluates every entry in full.
    sig^2 max|x|^2 stays below 96, so the kernel takes the norm expansion that
    the far path needs."""
    rng = np.random.default_rng(int(gap * 10))
    x = _two_caps(3000, gap)
    assert math.log2(math.e) / GAUSS[1] ** 2 * np.max(np.sum(x * x, axis=1)) < 96.0
    n, B = x.shape[0], 64
    q = rng.uniform(0.5, 1.5, size=n) * 0.5 / n
    U = rng.normal(0.2, 0.4, size=(B, n))
    theta = rng.uniform(0.15, 0.3, size=B)
    prob = P.Problem(ctx, torch.from_numpy(x).cuda(), torch.from_numpy(q).cuda())
    k = P.kernel_struct(NF.GAUSS_MH, *GAUSS)
    far, tot = prob.far_blocks(k)
    assert far > (0.3 if gap < 1.5 else 0.45) * tot, (far, tot)
    y = _apply(ctx, x, q, U, NF.GAUSS_MH, GAUSS, 20.0, theta, 4)
    ref = NF.apply_K(x, q, U, NF.GAUSS_MH, GAUSS, 20.0, theta)
    err = np.max(np.abs(y - ref) / _scale(x, q, U, NF.GAUSS_MH, GAUSS, 20.0, theta))
    print("fused form 4, two caps %.1f apart: %.2f of blocks far, max |dy| / S = %.3e" % (gap, far / tot, err),
          flush=True)
    assert err <= TOL_APPLY[4], err


def test_fused_tile_order_checkpoints_and_resume(ctx):
    """The fused BF16 form steps the states in the problem's tile order: every
    checkpoint comes back in the caller's node order (against the oracle's
    states at the same steps), and resuming from a checkpoint reproduces the
    uninterrupted run bit for bit."""
    w = C.ellipsoid_ensemble(2000, 64, steps=6)
    q = Q.surface_weights(w.surface)
    op = NF.DenseOperator(w.surface.xyz, q, w.kernel_kind, w.kernel)
    _, saved = NF.rk4(op, w.u0, w.beta, w.theta, w.dt, w.steps, save_every=2)
    prob = P.Problem(ctx, torch.from_numpy(w.surface.xyz).cuda(), torch.from_numpy(q).cuda())
    k = P.kernel_struct(w.kernel_kind, *w.kernel)
    f = P.Firing(w.beta, torch.from_numpy(w.theta).cuda())
    assert prob.far_blocks(k)[0] > 0
    u = torch.from_numpy(w.u0.copy()).cuda()
    ck = prob.integrate(k, f, u, w.dt, w.steps, form=4, ckpt_every=2)
    torch.cuda.synchronize()
    ck = ck.cpu().numpy()
    assert ck.shape == (4, 64, w.n)
    for i, ref in enumerate(saved):
        err = NF.rel_linf(ck[i], ref)
        assert np.all(err <= TOL_STATE[4]), (i, err.max())
    np.testing.assert_array_equal(ck[-1], u.cpu().numpy())
    u2 = torch.from_numpy(ck[1].copy()).cuda()    # resume from step 2
    prob.integrate(k, f, u2, w.dt, 4, form=4)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(u2.cpu().numpy(), u.cpu().numpy())
