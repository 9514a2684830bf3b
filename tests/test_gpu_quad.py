"""GPU surface quadrature weights (nfr_quad_weights) against the FP64 oracle.

* stencils: an integer result decided by FP64 squared distances that both
  sides evaluate in the same order without fused multiply-add: bit-exact;
* projection points: the same 3 x 3 solves, to 1e-12 of the surface's size;
* weights: both sides solve the same saddle-point systems in FP64 with LU and
  partial pivoting, in different operation orders (and different log / sqrt
  implementations); the systems' condition numbers (up to about 1e6 for r^3 on
  unit-scaled stencils) amplify rounding differences of 1e-16 to at most
  ~1e-10 of max|q|, the tolerance used here (observed: 3e-13 on the
  ellipsoid, 3e-12 on the torus at N = 65536).
"""
import numpy as np
import pytest
import torch

from oracle import quadrature as Q
from workloads import configs as C
from workloads import meshes
from workloads import surfaces as S

pytestmark = pytest.mark.gpu
P = pytest.importorskip("paper_2504_13379_amd")
TOL = 1e-10


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return P.Context(0)


def _gpu(ctx, surf, k, tris=None):
    tris = meshes.triangulate(surf) if tris is None else tris
    q, st, pj = P.quad_weights(ctx, torch.from_numpy(surf.xyz), torch.from_numpy(surf.normals), tris,
                               surf.star_shaped, k, details=True)
    torch.cuda.synchronize()
    return tris, q.cpu().numpy(), st.cpu().numpy(), pj.cpu().numpy()


@pytest.mark.parametrize("kind,n,k", [("sphere", 1500, 32), ("ellipsoid", 3001, 32), ("bumpy", 2500, 21),
                                      ("torus", 3000, 32), ("torus", 1200, 12), ("sphere", 700, 57)])
def test_quad_weights_match_oracle(ctx, kind, n, k):
    surf = S.make_surface(kind, n, np.random.default_rng(n))
    tris, q, st, pj = _gpu(ctx, surf, k)
    x = surf.xyz
    a, b, c = x[tris[:, 0]], x[tris[:, 1]], x[tris[:, 2]]
    cen = (a + b + c) / 3.0
    assert np.array_equal(st, Q.stencils(x, cen, k))
    p_ref, n_orth = Q.projection_points(surf, tris)
    assert np.array_equal(np.isnan(pj[:, 0]), np.isnan(p_ref[:, 0]))
    ok = ~np.isnan(p_ref[:, 0])
    assert np.max(np.abs(pj[ok] - p_ref[ok])) <= 1e-12 * max(1.0, np.max(np.abs(p_ref[ok])))
    q_ref = Q.surface_weights(surf, k=k)
    err = np.max(np.abs(q - q_ref)) / np.max(np.abs(q_ref))
    assert err <= TOL, err


def test_quad_weights_deterministic_and_reused_triangles(ctx):
    surf = S.torus(2000, np.random.default_rng(3))
    tris = meshes.triangulate(surf)
    _, q1, _, _ = _gpu(ctx, surf, 32, tris)
    _, q2, _, _ = _gpu(ctx, surf, 32, tris.copy())
    assert np.array_equal(q1, q2)


def test_quad_weights_full_size_ellipsoid(ctx):
    """The ellipsoid ensemble's surface at full size (N = 65536, 131068 triangles)."""
    surf = S.ellipsoid(65536)
    _, q, st, _ = _gpu(ctx, surf, 32)
    q_ref = Q.surface_weights(surf, k=32)
    assert np.max(np.abs(q - q_ref)) / np.max(np.abs(q_ref)) <= TOL
    assert abs(q.sum() - C.surface_area(surf)) <= 1e-6 * C.surface_area(surf)


@pytest.mark.parametrize("kind,n", [("torus", 3000), ("ellipsoid", 2500), ("sphere", 1500)])
def test_quad_weights_orthogonal_projection_match_oracle(ctx, kind, n):
    """Every triangle projected orthogonally along its normal (p_j at infinity,
    Jacobian 1 / |n(x) . n_j|): the branch the cutting-plane path takes only
    for singular systems, forced for all triangles on both sides."""
    surf = S.make_surface(kind, n, np.random.default_rng(n))
    tris = meshes.triangulate(surf)
    q, st, pj = P.quad_weights(ctx, torch.from_numpy(surf.xyz), torch.from_numpy(surf.normals), tris,
                               P.PROJ_ORTHOGONAL, 32, details=True)
    torch.cuda.synchronize()
    q, pj = q.cpu().numpy(), pj.cpu().numpy()
    assert np.all(np.isnan(pj))
    q_ref, info = Q.surface_weights(surf, k=32, projection="orthogonal", return_info=True)
    assert info["orthogonal_fallbacks"] == tris.shape[0]
    err = np.max(np.abs(q - q_ref)) / np.max(np.abs(q_ref))
    assert err <= TOL, err


def test_quad_weights_rejects_unknown_projection(ctx):
    surf = S.sphere(200)
    with pytest.raises(P.NfrError):
        P.quad_weights(ctx, torch.from_numpy(surf.xyz), torch.from_numpy(surf.normals), meshes.triangulate(surf), 3)
