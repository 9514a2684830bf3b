"""Pins for the oracle's surface RBF quadrature weights (CPU only).

Each check compares against mathematics fixed independently of the oracle:
closed-form surface integrals (the paper's sphere and torus test functions,
Gamma-function moments), an independent Duffy/Gauss-Legendre integrator,
exactness properties of the RBF-QF element solve, Euler characteristics, and
the paper's convergence claim (at least O(n^{-deg/2}) for degree deg).
"""
import math

import numpy as np
import pytest

from oracle import quadrature as Q
from tests import pins
from workloads import configs as C
from workloads import surfaces as S


def _rng(seed=0):
    return np.random.default_rng(seed)


# ---------------------------------------------------------------- building blocks


@pytest.mark.parametrize("seed", range(6))
def test_r3_triangle_closed_form_matches_duffy_rule(seed):
    rng = _rng(seed)
    v = rng.uniform(-1, 1, size=(3, 2))
    for P in [rng.uniform(-1.5, 1.5, size=2), v.mean(axis=0), v[0].copy(), 0.5 * (v[0] + v[1])]:
        exact = Q.r3_over_triangle(P, v[0], v[1], v[2])
        ref = pins.triangle_integral(lambda s: np.linalg.norm(s - P, axis=-1) ** 3,
                                     v[0], v[1], v[2], P=P, n=48)
        assert abs(exact - ref) <= 1e-12 * max(1.0, abs(ref))


def test_r3_apex_triangle_far_outside_point():
    # point far along the extension of an edge: angles close to +-pi/2
    v0, v1, v2 = np.array([0.0, 0.0]), np.array([1.0, 0.0]), np.array([0.3, 0.7])
    P = np.array([25.0, 1e-6])
    exact = Q.r3_over_triangle(P, v0, v1, v2)
    ref = pins.triangle_integral(lambda s: np.linalg.norm(s - P, axis=-1) ** 3, v0, v1, v2, P=P, n=48)
    assert abs(exact - ref) <= 1e-11 * abs(ref)


def test_monomial_integrals_match_duffy_rule():
    rng = _rng(7)
    v = rng.uniform(-1, 1, size=(3, 2))
    got = Q.monomial_integrals_deg2(v[0], v[1], v[2])
    ref = [pins.triangle_integral(lambda s, m=m: Q.monomials_deg2(s)[..., m], v[0], v[1], v[2])
           for m in range(6)]
    np.testing.assert_allclose(got, ref, rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("seed", range(4))
def test_element_rule_is_exact_on_its_interpolation_space(seed):
    """For f = sum_r c_r |s - s_r|^3 + poly (with Pi^T c = 0) the element rule is exact."""
    rng = _rng(100 + seed)
    k = 32
    v = np.array([[0.0, 0.0], [0.3, 0.0], [0.1, 0.28]]) + rng.normal(0, 0.02, size=(3, 2))
    s = rng.uniform(-0.5, 0.8, size=(k, 2))
    w = Q.planar_element_weights(s, v[0], v[1], v[2])
    Pi = Q.monomials_deg2(s)
    c = rng.normal(size=k)
    c -= Pi @ np.linalg.lstsq(Pi, c, rcond=None)[0]          # moment conditions Pi^T c = 0
    d = rng.normal(size=6)

    def f(pts):
        r = np.linalg.norm(pts[..., None, :] - s, axis=-1)
        return (r ** 3) @ c + Q.monomials_deg2(pts) @ d
    exact = pins.triangle_integral(f, v[0], v[1], v[2], n=48)
    rule = float(w @ f(s))
    assert abs(rule - exact) <= 1e-10 * max(1.0, abs(exact))


def test_element_rule_reproduces_polynomials():
    rng = _rng(3)
    s = rng.uniform(-1, 1, size=(21, 2))
    v = np.array([[-0.2, -0.2], [0.3, -0.1], [0.0, 0.35]])
    w = Q.planar_element_weights(s, v[0], v[1], v[2])
    for m in range(6):
        ref = pins.triangle_integral(lambda p, m=m: Q.monomials_deg2(p)[..., m], v[0], v[1], v[2])
        assert abs(w @ Q.monomials_deg2(s)[:, m] - ref) < 1e-12


def test_stencils_are_nearest_with_index_tiebreak():
    x = np.array([[1.0, 0, 0], [-1.0, 0, 0], [0, 1.0, 0], [0, -1.0, 0], [0, 0, 3.0]])
    st = Q.stencils(x, np.zeros((1, 3)), 4)
    assert st.tolist() == [[0, 1, 2, 3]]


def test_stencils_match_plain_loop_ranking_with_many_ties():
    """A jittered cloud plus an integer lattice whose centres sit on lattice
    points (every ring of equidistant nodes is an exact tie): the stencils equal
    a pure-Python ranking by (((dx*dx) + dy*dy) + dz*dz, index)."""
    rng = _rng(4)
    g = np.arange(-6, 7, dtype=np.float64)
    gx, gy = np.meshgrid(g, g, indexing="ij")
    lattice = np.stack([gx.ravel(), gy.ravel(), np.zeros(gx.size)], axis=1)
    cloud = rng.normal(size=(200, 3)) * 4.0
    # 30 integer points at squared distance exactly 25 from (100, 100, 100): more
    # ties than the k-d tree's proposals, so the full-scan ranking is exercised
    shell = [p for p in {(sx * a, sy * b, sz * c) for a, b, c in ((3, 4, 0), (4, 3, 0), (0, 3, 4), (0, 4, 3), (3, 0, 4),
                                                              (4, 0, 3), (5, 0, 0), (0, 5, 0), (0, 0, 5))
                         for sx in (-1, 1) for sy in (-1, 1) for sz in (-1, 1)}]
    shell = 100.0 + np.array(sorted(shell), dtype=np.float64)
    assert len(shell) == 30
    x = np.concatenate([cloud, lattice, shell])
    centres = np.concatenate([lattice[rng.choice(len(lattice), 10, replace=False)], rng.normal(size=(10, 3)),
                              np.full((1, 3), 100.0)])
    for k in (6, 21, 32):
        st = Q.stencils(x, centres, k)
        for c, row in zip(centres, st):
            def key(j):
                dx, dy, dz = x[j, 0] - c[0], x[j, 1] - c[1], x[j, 2] - c[2]
                return ((dx * dx + dy * dy) + dz * dz, j)
            assert row.tolist() == sorted(range(len(x)), key=key)[:k]


# ---------------------------------------------------------------- triangulations


@pytest.mark.parametrize("kind,chi", [("sphere", 2), ("ellipsoid", 2), ("bumpy", 2), ("torus", 0)])
def test_triangulation_is_closed_oriented_surface(kind, chi):
    surf = S.make_surface(kind, 3000, _rng(1))
    tris = Q.triangulate(surf)
    directed = np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]])
    # consistently oriented closed surface: every directed edge once, its reverse once
    keys = set(map(tuple, directed.tolist()))
    assert len(keys) == directed.shape[0]
    assert all((b, a) in keys for a, b in keys)
    n_edges = directed.shape[0] // 2
    assert surf.n - n_edges + tris.shape[0] == chi
    assert np.unique(tris).size == surf.n


# ---------------------------------------------------------------- surface rules


@pytest.fixture(scope="module")
def sphere_rules():
    out = {}
    for n in (1000, 4000, 16000):
        s = S.sphere(n)
        out[n] = (s, Q.surface_weights(s))
    return out


def test_sphere_paper_test_functions(sphere_rules):
    s, q = sphere_rules[16000]
    x, y, z = s.xyz.T
    # paper's sphere test functions: 1, x^3 y^2 z^4 + 5 (integral 20 pi), sin x cos 2y cos 3z (0)
    assert abs(q.sum() - 4 * math.pi) < 1e-6 * 4 * math.pi
    assert abs(q @ (x ** 3 * y ** 2 * z ** 4 + 5) - 20 * math.pi) < 1e-6 * 20 * math.pi
    assert abs(q @ (np.sin(x) * np.cos(2 * y) * np.cos(3 * z))) < 1e-7
    # weight-sign diagnostic sum(q) - sum|q|
    assert q.sum() - np.abs(q).sum() > -1e-3


@pytest.mark.parametrize("abc", [(2, 0, 0), (2, 2, 0), (0, 0, 4), (2, 2, 2), (4, 2, 0), (1, 0, 0), (1, 1, 1), (3, 0, 2)])
def test_sphere_monomial_moments(sphere_rules, abc):
    s, q = sphere_rules[16000]
    x, y, z = s.xyz.T
    a, b, c = abc
    assert abs(q @ (x ** a * y ** b * z ** c) - pins.sphere_monomial_integral(a, b, c)) < 1e-5


def test_sphere_convergence_rate(sphere_rules):
    errs = [abs(sphere_rules[n][1] @ (np.exp(sphere_rules[n][0].xyz[:, 0])) -
                2 * math.pi * (math.e - 1 / math.e)) for n in (1000, 4000, 16000)]
    # deg = 2 promises at least O(n^{-1}); a 4x refinement must cut the error >= 4x
    assert errs[1] < errs[0] / 4 and errs[2] < errs[1] / 4


@pytest.fixture(scope="module")
def torus_rules():
    out = {}
    for n in (4000, 16000):
        s = S.torus(n, _rng(1))
        out[n] = (s, Q.surface_weights(s, return_info=True))
    return out


def test_torus_paper_test_function_and_rate(torus_rules):
    R, r = 1.0, 0.4
    exact = 4 * math.pi ** 2 * R * r          # sin(7x) integrates to zero by symmetry phi -> pi - phi
    errs = []
    for n in (4000, 16000):
        s, (q, info) = torus_rules[n]
        assert info["orthogonal_fallbacks"] == 0
        errs.append(abs(q @ (np.sin(7 * s.xyz[:, 0]) + 1) - exact))
    assert errs[1] < 2e-4 * exact
    assert errs[1] < errs[0] / 4


def test_torus_second_moment(torus_rules):
    s, (q, _) = torus_rules[16000]
    R, r = 1.0, 0.4
    # int z^2 dA = int r^2 sin^2(t) r (R + r cos t) dt dphi = 2 pi^2 R r^3
    assert abs(q @ s.xyz[:, 2] ** 2 - 2 * math.pi ** 2 * R * r ** 3) < 1e-5


def test_ellipsoid_area_formula_matches_numeric():
    assert abs(C.ellipsoid_area(1.0, 0.8, 0.6) - pins.ellipsoid_area_numeric(1.0, 0.8, 0.6)) < 1e-10


@pytest.mark.parametrize("kind", ["ellipsoid", "bumpy"])
def test_star_shaped_surface_area(kind):
    s = S.make_surface(kind, 8000, _rng(0))
    q = Q.surface_weights(s)
    area = C.surface_area(s)
    assert abs(q.sum() - area) < 2e-5 * area


def test_bumpy_area_rule_converged():
    assert abs(C.bumpy_area(200, 400) - C.bumpy_area(300, 600)) < 1e-12


# ---------------------------------------------------------------- one element against its curved patch


@pytest.mark.parametrize("kind,projection", [("ellipsoid", "auto"), ("ellipsoid", "orthogonal"),
                                             ("torus", "auto"), ("torus", "orthogonal")])
def test_element_rule_integrates_its_curved_patch(kind, projection):
    """Section 3.3, eq. integral: one element's weights integrate over the curved
    patch that the projection (central from p_j, or orthogonal along n_j) maps
    onto E_j.  The reference integral comes from the definition of the area
    element (surface point on the projection line by Newton on the level set,
    |dx/ds1 x dx/ds2| by central differences, Duffy Gauss-Legendre over E_j),
    so it shares neither the pre-image nor the Jacobian formula with the oracle.

    Discrimination: dropping J turns the element rule for f = 1 into the flat
    triangle's area, an error of |patch - flat|; the test demands ten times
    less.  f = 1 + xy + sin 3z catches a wrong pre-image (wrong nodes weighted).
    """
    n = 16000
    surf = S.ellipsoid(n, (1.0, 0.8, 0.6)) if kind == "ellipsoid" else S.torus(n, _rng(7), 1.0, 0.4)
    F, G = pins.implicit_surface(kind, surf.params)
    x, nrm = surf.xyz, surf.normals
    tris = Q.triangulate(surf)
    P, n_orth = Q.projection_points(surf, tris, projection=projection)
    assert n_orth == (tris.shape[0] if projection == "orthogonal" else 0)
    pick = _rng(11).choice(tris.shape[0], 12, replace=False)
    a, b, c = x[tris[pick, 0]], x[tris[pick, 1]], x[tris[pick, 2]]
    st = Q.stencils(x, (a + b + c) / 3, 32)
    wE = Q.element_weights(x, nrm, a, b, c, P[pick], st)

    def fun(X):
        return 1.0 + X[..., 0] * X[..., 1] + np.sin(3 * X[..., 2])

    def one(X):
        return np.ones(X.shape[:-1])
    for j in range(len(pick)):
        pj = None if projection == "orthogonal" else P[pick[j]]
        area = pins.patch_integral(one, F, G, a[j], b[j], c[j], pj)
        flat = 0.5 * np.linalg.norm(np.cross(b[j] - a[j], c[j] - a[j]))
        err1 = abs(wE[j].sum() - area)
        assert err1 <= 0.1 * abs(area - flat) and err1 <= 2e-5 * area, (j, err1, area - flat)
        ref = pins.patch_integral(fun, F, G, a[j], b[j], c[j], pj)
        assert abs(wE[j] @ fun(x[st[j]]) - ref) <= 2e-4 * abs(ref), j


# ---------------------------------------------------------------- orthogonal projection everywhere


@pytest.fixture(scope="module")
def orthogonal_rules():
    out = {}
    for n in (1000, 4000, 16000):
        s = S.sphere(n)
        t = S.torus(n, _rng(7), 1.0, 0.4)
        out[n] = ((s, Q.surface_weights(s, projection="orthogonal", return_info=True)),
                  (t, Q.surface_weights(t, projection="orthogonal", return_info=True)))
    return out


def test_orthogonal_rule_paper_test_functions_and_rate(orthogonal_rules):
    """Every triangle projected orthogonally (p_j at infinity along n_j): the
    patches of neighbouring elements overlap or leave slivers of width
    O(h^3) along each edge, so the rule converges at O(h^2) = O(1/N), the
    rate deg = 2 promises.  Sphere: 1 -> 4 pi, x^3 y^2 z^4 + 5 -> 20 pi;
    torus: sin(7x) + 1 -> 4 pi^2 R r.  Error >= 3.5x smaller per 4x nodes."""
    sph, tor = [], []
    for n in (1000, 4000, 16000):
        (s, (qs, info_s)), (t, (qt, info_t)) = orthogonal_rules[n]
        assert info_s["orthogonal_fallbacks"] == info_s["triangles"]
        assert info_t["orthogonal_fallbacks"] == info_t["triangles"]
        x, y, z = s.xyz.T
        sph.append(max(abs(qs.sum() - 4 * math.pi) / (4 * math.pi),
                       abs(qs @ (x ** 3 * y ** 2 * z ** 4 + 5) - 20 * math.pi) / (20 * math.pi)))
        area = 4 * math.pi ** 2 * 0.4
        tor.append(abs(qt @ (np.sin(7 * t.xyz[:, 0]) + 1) - area) / area)
    assert sph[2] < 3e-4 and tor[2] < 4e-4, (sph, tor)
    assert sph[1] < sph[0] / 3.5 and sph[2] < sph[1] / 3.5, sph
    assert tor[1] < tor[0] / 3.5 and tor[2] < tor[1] / 3.5, tor
