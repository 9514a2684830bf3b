"""RBF quadrature weights on closed surfaces (FP64 CPU oracle; test infrastructure).

This module is part of the correctness oracle.  Only the test-suite, the smoke
check and the CPU-baseline leg of the benchmark may import it; the GPU library
never does.

It computes surface quadrature weights q with Q_n f = sum_i q_i f(x_i), the
``mu_j`` of the discrete collocation scheme (paper section 2.2, eq.
NFODETilde), following the paper's section 3:

* local interpolation with the polyharmonic spline r^3 plus polynomials of
  degree <= deg on stencils of the k nodes nearest to an element's centre
  (section 3.1, eqs. polyHarmonic and interp_system);
* RBF-QF for the integral functional: per element, the weights solve the
  saddle-point system with right-hand side the exact integrals of the basis
  functions over the element, and a node's weight is the sum of its
  element weights (section 3.2, eq. functional_stencil);
* on a curved surface, the flat triangles E_j are mapped to curved patches by
  central projection from projection points p_j; each stencil is pulled back
  to the plane of E_j along rays through p_j, planar RBF-QF is applied there,
  and the Jacobian of the map multiplies each weight (section 3.3, eq.
  integral).

Readings where the paper is silent or garbled:

* the cutting plane of an edge shared by E_j and E_j' contains that edge and
  has normal n_j - n_j' (the printed condition drops the edge point);
* star-shaped surfaces use p_j = 0 for every triangle: every plane through the
  origin and an edge is shared by both neighbours, so the curved patches
  partition the surface exactly;
* where the three cutting planes of a torus triangle are nearly parallel
  (zero Gaussian curvature), the projection is taken orthogonally onto the
  triangle's plane (p_j at infinity along n_j);
* the Jacobian that eq. integral carries is applied to the planar weights,
  evaluated at each stencil node's pre-image;
* stencil ties are broken by (distance, index).

Flat domains (the squares of the paper's section 4) use the planar rule of
section 3.2 directly: a Delaunay triangulation of the nodes, the same stencils
and element weights, no projection and no Jacobian.
"""
from __future__ import annotations

import numpy as np
from scipy.spatial import Delaunay, cKDTree

from workloads import meshes

# ------------------------------------------------------------- triangulation

# The flat triangulation {E_j} (section 3.3: a planar triangulation whose
# vertices are the nodes) is an input of the method, built with the node sets
# in workloads/meshes.py; it is re-exported here for the oracle's callers.
triangulate = meshes.triangulate


def edges_of(tris: np.ndarray):
    """Unique undirected edges and, for every triangle edge, the other triangle."""
    m = tris.shape[0]
    e = np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]])  # (3m, 2)
    owner = np.concatenate([np.arange(m)] * 3)
    key = np.sort(e, axis=1)
    order = np.lexsort((key[:, 1], key[:, 0]))
    ks = key[order]
    same = np.all(ks[1:] == ks[:-1], axis=1)
    neighbour = np.full(3 * m, -1, dtype=np.int64)
    i = np.nonzero(same)[0]
    neighbour[order[i]] = owner[order[i + 1]]
    neighbour[order[i + 1]] = owner[order[i]]
    uniq = np.unique(key, axis=0)
    return uniq, neighbour.reshape(3, m).T   # neighbour[j, e]: across edge e of triangle j


# ------------------------------------------------- exact integrals on a triangle


def _log_rho_plus_l(rho, l, d):
    """log(rho + l) with rho = sqrt(d^2 + l^2); for l < 0 uses rho + l = d^2 / (rho - l)."""
    with np.errstate(divide="ignore", invalid="ignore"):
        pos = np.log(np.where(l >= 0, rho + l, 1.0))
        neg = 2.0 * np.log(np.where(l < 0, d, 1.0)) - np.log(np.where(l < 0, rho - l, 1.0))
    return np.where(l >= 0, pos, neg)


def _safe_diff(d, a, b):
    with np.errstate(invalid="ignore"):
        return np.where(d > 0, a - b, 0.0)


def r3_over_apex_triangle(P, p, q):
    """Integral of |s - P|^3 over the triangle (P, p, q), unsigned (2-D points).

    In polar coordinates about P, with d the distance from P to the line pq and
    alpha the angle from the foot of the perpendicular,
      int = (d^5 / 5) [S(alpha)]  with  S = int sec^5 = sec^3 tan / 4
            + 3 sec tan / 8 + 3 ln(sec + tan) / 8,
    written with rho = d sec(alpha) and l = d tan(alpha) so that d = 0 is safe:
      int = (d / 5) [ rho^3 l / 4 + 3 d^2 rho l / 8 + 3 d^4 ln(rho + l) / 8 ].
    Arrays broadcast over leading dimensions; the last axis has length 2.
    """
    t = q - p
    L = np.linalg.norm(t, axis=-1)
    t = t / L[..., None]
    lp = np.sum((p - P) * t, axis=-1)           # signed position of p along t, from the foot
    lq = lp + L
    d = np.abs((p - P)[..., 0] * t[..., 1] - (p - P)[..., 1] * t[..., 0])
    rp = np.sqrt(d * d + lp * lp)
    rq = np.sqrt(d * d + lq * lq)
    d2 = d * d
    term = (0.25 * (rq ** 3 * lq - rp ** 3 * lp)
            + 0.375 * d2 * (rq * lq - rp * lp)
            + 0.375 * d2 * d2 * _safe_diff(d, _log_rho_plus_l(rq, lq, d), _log_rho_plus_l(rp, lp, d)))
    return d * term / 5.0


def r3_over_triangle(P, v0, v1, v2):
    """Integral of |s - P|^3 over triangle (v0, v1, v2) for points P (..., 2).

    Signed decomposition into the three triangles with apex P: each apex
    triangle counts with the sign of its orientation relative to the triangle's.
    """
    def cross2(a, b):
        return a[..., 0] * b[..., 1] - a[..., 1] * b[..., 0]
    o = np.sign(cross2(v1 - v0, v2 - v0))
    total = 0.0
    for p, q in ((v0, v1), (v1, v2), (v2, v0)):
        s = np.sign(cross2(p - P, q - P)) * o
        total = total + s * r3_over_apex_triangle(P, p, q)
    return total


def monomials_deg2(s):
    """Polynomial basis of degree <= 2 in 2-D: 1, x, y, x^2, x y, y^2."""
    x, y = s[..., 0], s[..., 1]
    return np.stack([np.ones_like(x), x, y, x * x, x * y, y * y], axis=-1)


def monomial_integrals_deg2(v0, v1, v2):
    """Exact integrals of the degree-2 basis over a triangle (edge-midpoint rule)."""
    area = 0.5 * np.abs((v1 - v0)[..., 0] * (v2 - v0)[..., 1] - (v1 - v0)[..., 1] * (v2 - v0)[..., 0])
    mids = ((v0 + v1) / 2, (v1 + v2) / 2, (v2 + v0) / 2)
    acc = sum(monomials_deg2(m) for m in mids)
    return acc * (area / 3.0)[..., None]


# -------------------------------------------------------------- projection


def projection_points(surface, tris, cond_max: float = 1e8, projection: str = "auto"):
    """p_j for every triangle, or NaN rows meaning "at infinity along n_j".

    projection="auto": star-shaped surfaces use the origin; other surfaces the
    intersection of the three cutting planes {y : (n_j - n_j') . (y - a_e) = 0},
    one per edge e shared with neighbour j'; if those planes are nearly
    parallel (condition number above cond_max) the triangle falls back to
    orthogonal projection.  projection="orthogonal": every triangle projects
    orthogonally onto its own plane (section 3.3 allows p_j at infinity).
    Returns (P, number of orthogonal rows).
    """
    m = tris.shape[0]
    if projection == "orthogonal":
        return np.full((m, 3), np.nan), m
    if projection != "auto":
        raise ValueError("projection must be 'auto' or 'orthogonal'")
    if surface.star_shaped:
        return np.zeros((m, 3)), 0
    x = surface.xyz
    a, b, c = x[tris[:, 0]], x[tris[:, 1]], x[tris[:, 2]]
    nj = np.cross(b - a, c - a)
    nj /= np.linalg.norm(nj, axis=1, keepdims=True)
    _, nb = edges_of(tris)
    if np.any(nb < 0):
        raise ValueError("triangulation is not closed")
    M = nj[:, None, :] - nj[nb]                       # (m, 3, 3): rows are cutting-plane normals
    M /= np.linalg.norm(M, axis=2, keepdims=True)
    ea = np.stack([a, b, c], axis=1)                  # a point on each edge (edge e starts at vertex e)
    cen = (a + b + c) / 3.0
    rhs = np.sum(M * (ea - cen[:, None, :]), axis=2)
    sv = np.linalg.svd(M, compute_uv=False)
    cond = sv[:, 0] / np.maximum(sv[:, 2], 1e-300)
    ok = cond <= cond_max
    p = np.full((m, 3), np.nan)
    p[ok] = cen[ok] + np.linalg.solve(M[ok], rhs[ok][..., None])[..., 0]
    return p, int(np.count_nonzero(~ok))


# -------------------------------------------------------------- weights


def planar_element_weights(s2, v0, v1, v2):
    """RBF-QF weights of one flat element for its (planar) stencil.

    s2: (..., k, 2) stencil points; v0, v1, v2: (..., 2) triangle vertices.
    Solves [A Pi; Pi^T 0][w; gamma] = [int_E |s - s_r|^3 ds ; int_E pi(s) ds]
    with A_rs = |s_r - s_s|^3 and Pi the degree-2 monomials, and returns w.
    """
    k = s2.shape[-2]
    mpoly = 6
    kk = k + mpoly
    lead = s2.shape[:-2]
    diff = s2[..., :, None, :] - s2[..., None, :, :]
    Amat = np.linalg.norm(diff, axis=-1) ** 3
    Pi = monomials_deg2(s2)
    sysm = np.zeros(lead + (kk, kk))
    sysm[..., :k, :k] = Amat
    sysm[..., :k, k:] = Pi
    sysm[..., k:, :k] = np.swapaxes(Pi, -1, -2)
    rhs = np.empty(lead + (kk,))
    rhs[..., :k] = r3_over_triangle(s2, v0[..., None, :], v1[..., None, :], v2[..., None, :])
    rhs[..., k:] = monomial_integrals_deg2(v0, v1, v2)
    sol = np.linalg.solve(sysm, rhs[..., None])[..., 0]
    return sol[..., :k]



def squared_distances(points: np.ndarray, centre: np.ndarray) -> np.ndarray:
    """|p - c|^2 summed over the coordinates in order, every operation an FP64
    rounding (no fused multiply-add): the exact quantity stencils are ranked by."""
    diff = points - centre
    acc = diff[..., 0] * diff[..., 0]
    for a in range(1, diff.shape[-1]):
        acc = acc + diff[..., a] * diff[..., a]
    return acc


def stencils(xyz: np.ndarray, centres: np.ndarray, k: int) -> np.ndarray:
    """The k nodes nearest to every centre (section 3.3), ordered by the pair
    (squared distance as `squared_distances` evaluates it, node index).

    A k-d tree proposes k + 8 candidates per centre; the ranking uses the exact
    FP64 squared distances above.  A centre whose k-th exact distance is not
    safely below the tree's last proposal is ranked over all nodes instead.
    """
    n = xyz.shape[0]
    if k > n:
        raise ValueError("stencil larger than the node set")
    m = min(n, k + 8)
    dist, idx = cKDTree(xyz).query(centres, k=m)
    idx = np.asarray(idx, dtype=np.int64).reshape(centres.shape[0], m)
    d2 = squared_distances(xyz[idx], centres[:, None, :])
    order = np.lexsort((idx, d2), axis=-1)
    idx = np.take_along_axis(idx, order, axis=1)
    d2 = np.take_along_axis(d2, order, axis=1)
    out = idx[:, :k].copy()
    if m < n:
        last = np.asarray(dist, dtype=np.float64).reshape(centres.shape[0], m)[:, -1]
        unsure = np.nonzero(d2[:, k - 1] >= last * last * (1.0 - 1e-12))[0]
        for c in unsure:
            full = squared_distances(xyz, centres[c])
            out[c] = np.lexsort((np.arange(n), full))[:k]
    return out


def element_weights(x, nrm_x, a, b, c, P, st):
    """Surface RBF-QF weights of a set of triangles E_j (section 3.3, eq. integral).

    x, nrm_x: (N, 3) nodes and their exact unit normals; a, b, c: (m, 3)
    vertices of each E_j, oriented outward; P: (m, 3) projection points (a NaN
    row: orthogonal projection along n_j); st: (m, k) stencils.  For every
    triangle the stencil is pulled back to the plane of E_j (along rays from
    p_j, or along n_j), expressed in a 2-D frame centred at the centroid and
    scaled by the stencil radius h_j, and the planar weights of eq.
    functional_stencil are multiplied by h_j^2 and by the Jacobian J of the
    map from E_j's plane to the surface at each stencil node:
      central projection:    J = (|x - p| / |xi - p|)^2 |n_j . u| / |n(x) . u|,
                             u = (x - p) / |x - p|;
      orthogonal projection: J = 1 / |n(x) . n_j|.
    Returns (m, k): the weight of stencil node r in triangle j.
    """
    cen = (a + b + c) / 3.0
    nj = np.cross(b - a, c - a)
    nj /= np.linalg.norm(nj, axis=1, keepdims=True)
    xs = x[st]                                   # (m, k, 3)
    ns = nrm_x[st]
    nn = nj[:, None, :]
    orth = np.isnan(P[:, 0])
    # pre-images on the plane of E_j
    xi = np.empty_like(xs)
    J = np.empty(xs.shape[:2])
    if np.any(~orth):
        pp = P[~orth][:, None, :]
        dxp = xs[~orth] - pp
        num = np.sum(nn[~orth] * (a[~orth][:, None, :] - pp), axis=2)
        den = np.sum(nn[~orth] * dxp, axis=2)
        t = num / den
        xi_c = pp + t[..., None] * dxp
        xi[~orth] = xi_c
        u = dxp / np.linalg.norm(dxp, axis=2, keepdims=True)
        ratio = np.linalg.norm(dxp, axis=2) / np.linalg.norm(xi_c - pp, axis=2)
        cos_plane = np.abs(np.sum(nn[~orth] * u, axis=2))
        cos_surf = np.abs(np.sum(ns[~orth] * u, axis=2))
        J[~orth] = ratio ** 2 * cos_plane / cos_surf
    if np.any(orth):
        h_off = np.sum(nn[orth] * (xs[orth] - a[orth][:, None, :]), axis=2)
        xi[orth] = xs[orth] - h_off[..., None] * nn[orth]
        cs = np.abs(np.sum(ns[orth] * nn[orth], axis=2))
        J[orth] = 1.0 / cs
    # local 2-D frame centred at the centroid, scaled by h_j
    e1 = b - a
    e1 /= np.linalg.norm(e1, axis=1, keepdims=True)
    e2 = np.cross(nj, e1)
    rel = xi - cen[:, None, :]
    h = np.max(np.linalg.norm(rel, axis=2), axis=1)
    s2 = np.stack([np.sum(rel * e1[:, None, :], axis=2),
                   np.sum(rel * e2[:, None, :], axis=2)], axis=2) / h[:, None, None]
    verts = [np.stack([np.sum((v - cen) * e1, axis=1),
                       np.sum((v - cen) * e2, axis=1)], axis=1) / h[:, None]
             for v in (a, b, c)]
    wplan = planar_element_weights(s2, verts[0], verts[1], verts[2])
    return wplan * (h * h)[:, None] * J


def surface_weights(surface, k: int = 32, deg: int = 2, chunk: int = 8192,
                    return_info: bool = False, projection: str = "auto"):
    """Surface RBF-QF weights q (length N) with phi(r) = r^3 and degree-deg polynomials.

    For every triangle E_j: pull the stencil S(E_j) back to the plane of E_j
    (along rays from p_j; with projection="orthogonal", or where the cutting
    planes are singular, along n_j), scale by h_j about the centroid, solve
      [A  Pi; Pi^T 0] [w; gamma] = [int_E r^3 ; int_E pi]
    and add w_r * h_j^2 * J_j(xi_r) to q at stencil node r (`element_weights`).
    """
    if deg != 2:
        raise ValueError("only deg = 2 is implemented")
    mpoly = 6
    if k < mpoly:
        raise ValueError("stencil too small: k >= C(deg + 2, 2) is required")
    x, nrm_x = surface.xyz, surface.normals
    n = x.shape[0]
    tris = triangulate(surface)
    m = tris.shape[0]
    P, n_orth = projection_points(surface, tris, projection=projection)
    a, b, c = x[tris[:, 0]], x[tris[:, 1]], x[tris[:, 2]]
    cen = (a + b + c) / 3.0
    st = stencils(x, cen, k)
    q = np.zeros(n)
    min_cos = np.inf
    for lo in range(0, m, chunk):
        sl = slice(lo, min(m, lo + chunk))
        wE = element_weights(x, nrm_x, a[sl], b[sl], c[sl], P[sl], st[sl])
        q += np.bincount(st[sl].ravel(), weights=wE.ravel(), minlength=n)
        min_cos = min(min_cos, _min_cos(x, nrm_x, a[sl], b[sl], c[sl], P[sl], st[sl]))
    if return_info:
        return q, {"triangles": m, "orthogonal_fallbacks": n_orth, "min_cos": min_cos,
                   "tris": tris}
    return q


def _min_cos(x, nrm_x, a, b, c, P, st):
    """Smallest |n(x) . direction of projection| over the stencils (diagnostic)."""
    nj = np.cross(b - a, c - a)
    nj /= np.linalg.norm(nj, axis=1, keepdims=True)
    xs, ns = x[st], nrm_x[st]
    orth = np.isnan(P[:, 0])
    out = np.inf
    if np.any(~orth):
        d = xs[~orth] - P[~orth][:, None, :]
        d /= np.linalg.norm(d, axis=2, keepdims=True)
        out = min(out, float(np.abs(np.sum(ns[~orth] * d, axis=2)).min()))
    if np.any(orth):
        out = min(out, float(np.abs(np.sum(ns[orth] * nj[orth][:, None, :], axis=2)).min()))
    return out


def plane_weights(xy: np.ndarray, k: int = 32, chunk: int = 8192, return_info: bool = False):
    """Planar RBF-QF weights (paper section 3.2, eq. functional_stencil) for a
    convex planar domain covered by the Delaunay triangulation of its nodes.

    xy: (N, 2) nodes (or (N, 3) with the plane z = const).  Per triangle E_j
    the stencil is the k nodes nearest to its centroid c_j; in coordinates
    (x - c_j) / h_j, h_j the stencil radius, the weights solve
      [A  Pi; Pi^T 0] [w; gamma] = [int_E r^3 ; int_E pi]
    and w_r h_j^2 is added to q at stencil node r.  Triangles with area below
    1e-14 of the domain's bounding box (collinear boundary nodes) are dropped.
    """
    xy = np.ascontiguousarray(np.asarray(xy, dtype=np.float64)[:, :2])
    n = xy.shape[0]
    if k < 6:
        raise ValueError("stencil too small: k >= 6 is required for degree 2")
    tris = Delaunay(xy).simplices
    a, b, c = xy[tris[:, 0]], xy[tris[:, 1]], xy[tris[:, 2]]
    area = 0.5 * np.abs((b - a)[:, 0] * (c - a)[:, 1] - (b - a)[:, 1] * (c - a)[:, 0])
    box = np.prod(xy.max(axis=0) - xy.min(axis=0))
    keep = area > 1e-14 * box
    tris, a, b, c = tris[keep], a[keep], b[keep], c[keep]
    m = tris.shape[0]
    cen = (a + b + c) / 3.0
    st = stencils(xy, cen, k)
    q = np.zeros(n)
    for lo in range(0, m, chunk):
        sl = slice(lo, min(m, lo + chunk))
        rel = xy[st[sl]] - cen[sl][:, None, :]
        h = np.max(np.linalg.norm(rel, axis=2), axis=1)
        s2 = rel / h[:, None, None]
        verts = [(v[sl] - cen[sl]) / h[:, None] for v in (a, b, c)]
        w = planar_element_weights(s2, verts[0], verts[1], verts[2]) * (h * h)[:, None]
        q += np.bincount(st[sl].ravel(), weights=w.ravel(), minlength=n)
    if return_info:
        return q, {"triangles": m, "tris": tris, "area": float(area[keep].sum())}
    return q
