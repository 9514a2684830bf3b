"""nfr_apply_noalloc (the operator with the library's fixed device scratch, for
callers that cannot allocate) against nfr_apply with a caller workspace.

Both run the same kernels with the same launch plan, so their outputs must be
equal bit for bit.  Two calls in a row, the second on a smaller problem: the
scratch keeps the first call's bytes, and the second result must not depend
on them.  A call whose scratch would exceed the fixed size is rejected on the
host before anything is enqueued.
"""
import numpy as np
import pytest
import torch

from workloads import configs as C
from workloads import surfaces as S

pytestmark = pytest.mark.gpu
P = pytest.importorskip("paper_2504_13379_amd")
from paper_2504_13379_amd import _lib as L  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return P.Context(0, torch.cuda.Stream())


def _case(ctx, surf, B, kind, kern, seed):
    rng = np.random.default_rng(seed)
    x = torch.from_numpy(surf.xyz).cuda()
    q = torch.from_numpy(C.area_share_weights(surf) * (1.0 + 0.1 * rng.uniform(-1, 1, surf.n))).cuda()
    prob = P.Problem(ctx, x, q)
    u = torch.from_numpy(rng.normal(0.2, 0.3, size=(B, surf.n))).cuda()
    theta = torch.from_numpy(rng.uniform(0.15, 0.3, size=B)).cuda()
    return prob, P.kernel_struct(kind, *kern), P.Firing(20.0, theta), u


def _both(ctx, prob, k, f, u, form, W=None):
    ref = prob.apply(k, f, u, form=form, W=W)
    out = torch.full_like(u, float("nan"))
    prob.apply_noalloc(k, f, u, out, form=form, W=W)
    ctx.stream.synchronize()
    return ref.cpu().numpy(), out.cpu().numpy()


@pytest.mark.parametrize("first,second", [
    # (surface, N, B, kernel kind, form) of the first and the second, smaller call
    (("torus", 20000, 1, 1, L.FORM_ONTHEFLY_FP32), ("sphere", 3001, 1, 0, L.FORM_ONTHEFLY_FP32)),
    (("ellipsoid", 4096, 64, 0, L.FORM_ONTHEFLY_BF16X3), ("sphere", 1500, 16, 0, L.FORM_ONTHEFLY_BF16X3)),
    (("ellipsoid", 9000, 8, 0, L.FORM_ONTHEFLY_FP32), ("torus", 2500, 3, 1, L.FORM_W_FP32)),
    (("sphere", 6000, 32, 0, L.FORM_ONTHEFLY_FP32_MFMA), ("ellipsoid", 700, 5, 0, L.FORM_W_FP16X3)),
])
def test_noalloc_equals_apply_on_two_calls(ctx, first, second):
    kern = {0: (1.0, 0.15, 0.5, 0.4), 1: (2.0, 0.1, 1.0, 0.3)}
    for seed, (kind, n, B, kk, form) in enumerate((first, second)):
        surf = S.make_surface(kind, n, np.random.default_rng(seed + 10))
        prob, k, f, u = _case(ctx, surf, B, kk, kern[kk], seed)
        W = prob.w_build(k, form) if form in (L.FORM_W_FP32, L.FORM_W_BF16X3, L.FORM_W_FP16X3) else None
        need = L.lib().nfr_apply_workspace_size(prob.handle, B, form)
        assert 0 < need <= L.NFR_APPLY_NOALLOC_MAX_BYTES
        print("noalloc case", kind, n, B, form, need, flush=True)
        ref, got = _both(ctx, prob, k, f, u, form, W)
        assert np.all(np.isfinite(ref))
        assert np.array_equal(ref, got), (kind, n, B, form, np.max(np.abs(ref - got)))


def test_noalloc_rejects_oversized_scratch(ctx):
    """N = 65536 with 64 states on the fused BF16 form needs 134 MB of FP32 partial
    sums: rejected with NFR_ERR_WORKSPACE before anything is enqueued."""
    surf = S.ellipsoid(65536)
    prob, k, f, u = _case(ctx, surf, 64, 0, (1.0, 0.15, 0.5, 0.4), 3)
    assert L.lib().nfr_apply_workspace_size(prob.handle, 64, L.FORM_ONTHEFLY_BF16X3) > L.NFR_APPLY_NOALLOC_MAX_BYTES
    out = torch.zeros_like(u)
    with pytest.raises(P.NfrError) as e:
        prob.apply_noalloc(k, f, u, out, form=L.FORM_ONTHEFLY_BF16X3)
    assert e.value.status == L.NFR_ERR_WORKSPACE
    ctx.stream.synchronize()
    assert float(out.abs().max()) == 0.0
