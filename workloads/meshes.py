"""Flat triangulations of the node sets (inputs of the surface quadrature).

The surface RBF-QF method starts from nodes and a planar triangulation whose
vertices are exactly those nodes (paper section 3.3).  The triangulation is
built here with the node sets: for star-shaped surfaces the convex hull of the
node directions, for the torus strips between consecutive node rings.  No step
of the quadrature method itself lives in this module.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.spatial import ConvexHull


def triangulate(surface) -> np.ndarray:
    """Flat triangulation {E_j} whose vertices are exactly the nodes.

    Star-shaped surfaces: convex hull of the node directions.  Torus: strips
    between consecutive node rings, closed in both angles.  Triangles are
    oriented so that (b - a) x (c - a) points along the outward normal.
    """
    x = surface.xyz
    if surface.star_shaped:
        u = x / np.linalg.norm(x, axis=1, keepdims=True)
        tris = ConvexHull(u).simplices.astype(np.int64)
    elif surface.kind == "torus":
        tris = _torus_strips(surface)
    else:
        raise ValueError("no triangulation for %s" % surface.kind)
    a, b, c = x[tris[:, 0]], x[tris[:, 1]], x[tris[:, 2]]
    nrm = np.cross(b - a, c - a)
    ref = surface.normal_at((a + b + c) / 3.0)
    flip = np.sum(nrm * ref, axis=1) < 0
    tris[flip] = tris[flip][:, [0, 2, 1]]
    return tris


def _torus_strips(surface) -> np.ndarray:
    ring = surface.ring
    phi = surface.angles[:, 0]
    n_rings = int(ring.max()) + 1
    members = []
    for k in range(n_rings):
        idx = np.nonzero(ring == k)[0]
        members.append(idx[np.argsort(phi[idx], kind="stable")])
    out = []
    two_pi = 2.0 * math.pi
    for k in range(n_rings):
        A = members[k]
        B = members[(k + 1) % n_rings]
        a_ang = phi[A]
        b_ang = phi[B]
        ma, mb = len(A), len(B)
        d = np.abs(np.angle(np.exp(1j * (b_ang - a_ang[0]))))
        j0 = int(np.argmin(d))
        b0 = b_ang[j0]
        if b0 - a_ang[0] > math.pi:
            b0 -= two_pi
        elif a_ang[0] - b0 > math.pi:
            b0 += two_pi
        sa = np.arange(ma + 1)
        A_u = a_ang[sa % ma] + two_pi * (sa // ma)
        tb = np.arange(mb + 1)
        jb = (j0 + tb) % mb
        B_u = b_ang[jb] + two_pi * ((j0 + tb) // mb) - b_ang[j0] + b0
        s = t = 0
        while s < ma or t < mb:
            if s < ma and (t == mb or A_u[s + 1] <= B_u[t + 1]):
                out.append((A[s % ma], A[(s + 1) % ma], B[jb[t]]))
                s += 1
            else:
                out.append((A[s % ma], B[jb[t + 1]], B[jb[t]]))
                t += 1
    return np.asarray(out, dtype=np.int64)


