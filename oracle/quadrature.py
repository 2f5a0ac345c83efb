"""Quadrature rules on triangles (oracle; test infrastructure only).

The paper does not state its rules.  Reading (rule set Q):
  * Q7: Radon's 7-point degree-5 rule - centroid with weight 9/40, and the two
    orbits (b, b, 1-2b) with b = (6 -+ sqrt 15)/21 and weights (155 -+ sqrt 15)/1200.
  * Q3: the 3-point degree-2 rule (2/3, 1/6, 1/6) and permutations, weights 1/3.
Weights are relative to the triangle area (they sum to 1).

Also: Gauss-Legendre nodes (numpy's leggauss as the primitive), composite rules
obtained by 4-to-1 subdivision, and the brute-force inner integrator used to pin
the closed-form static potentials: the source triangle is split at the
projection of the observation point into three triangles, each mapped by a
Duffy (collapsed) transform and integrated with geometrically graded composite
Gauss-Legendre in the radial direction.
"""
from __future__ import annotations

import math

import numpy as np


def q7():
    s = math.sqrt(15.0)
    a1 = (6.0 - s) / 21.0
    a2 = (6.0 + s) / 21.0
    w1 = (155.0 - s) / 1200.0
    w2 = (155.0 + s) / 1200.0
    bary = [(1 / 3, 1 / 3, 1 / 3),
            (a1, a1, 1 - 2 * a1), (a1, 1 - 2 * a1, a1), (1 - 2 * a1, a1, a1),
            (a2, a2, 1 - 2 * a2), (a2, 1 - 2 * a2, a2), (1 - 2 * a2, a2, a2)]
    w = [9.0 / 40.0] + [w1] * 3 + [w2] * 3
    return np.array(bary), np.array(w)


def q3():
    bary = [(2 / 3, 1 / 6, 1 / 6), (1 / 6, 2 / 3, 1 / 6), (1 / 6, 1 / 6, 2 / 3)]
    return np.array(bary), np.full(3, 1.0 / 3.0)


def subdivided(rule, level: int):
    """Composite rule: the reference triangle split 4-to-1 `level` times, `rule` on each piece."""
    bary, w = rule
    tris = [np.eye(3)]  # rows = barycentric coordinates of the corners
    for _ in range(level):
        nxt = []
        for c in tris:
            m01, m12, m20 = (c[0] + c[1]) / 2, (c[1] + c[2]) / 2, (c[2] + c[0]) / 2
            nxt += [np.array([c[0], m01, m20]), np.array([m01, c[1], m12]),
                    np.array([m20, m12, c[2]]), np.array([m01, m12, m20])]
        tris = nxt
    pts = np.concatenate([bary @ c for c in tris])
    ws = np.concatenate([w / len(tris) for _ in tris])
    return pts, ws


def points(vertices: np.ndarray, bary: np.ndarray) -> np.ndarray:
    """Map barycentric points onto triangles.  vertices: (..., 3, 3) -> (..., nq, 3)."""
    return np.einsum("qi,...ij->...qj", bary, vertices)


def gauss_legendre(n: int, a: float = 0.0, b: float = 1.0):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (b - a) * x + 0.5 * (b + a), 0.5 * (b - a) * w


def graded_intervals(rmax: float, scale: float, ratio: float = 4.0):
    """Breakpoints of [0, rmax], geometric with factor `ratio` on both sides of `scale`."""
    pts = {0.0, rmax}
    x = min(scale, rmax)
    while x > 1e-9 * rmax:
        pts.add(x)
        x /= ratio
    x = min(scale, rmax) * ratio
    while x < rmax:
        pts.add(x)
        x *= ratio
    return sorted(pts)


def brute_inner(fun, r: np.ndarray, tri_xyz: np.ndarray, order: int = 24):
    """Integral over the flat triangle tri_xyz (3x3) of fun(rp) dS', robust to a
    singularity at the projection of r onto the triangle's plane.

    fun maps an (n, 3) array of source points to an (n, ...) array.  The triangle
    is split at the projection p into three triangles (p, v_i, v_{i+1}); each is
    parametrised by radius fraction s in [0, 1] along the ray from p and an edge
    parameter u in [0, 1], with dS' = 2 A_i s ds du; s is integrated with composite
    Gauss-Legendre refined geometrically towards s = 0 and u with composite
    Gauss-Legendre refined geometrically towards the foot of p on the edge.
    """
    v = np.asarray(tri_xyz, dtype=np.float64)
    n = np.cross(v[1] - v[0], v[2] - v[0])
    n /= np.linalg.norm(n)
    p = r - n * ((r - v[0]) @ n)
    d = abs((r - v[0]) @ n)
    total = 0.0
    for i in range(3):
        a, b = v[i], v[(i + 1) % 3]
        area2 = np.linalg.norm(np.cross(a - p, b - p))  # = 2 * area of (p, a, b), signed below
        sgn = np.sign(np.cross(a - p, b - p) @ n)
        if area2 < 1e-300:
            continue
        rmax = max(np.linalg.norm(a - p), np.linalg.norm(b - p))
        br = graded_intervals(1.0, max(d, 1e-3 * rmax) / rmax)
        # angular grading around the foot of p on the edge (thin fan triangles)
        L = np.linalg.norm(b - a)
        u0 = float(np.clip((p - a) @ (b - a) / (L * L), 0.0, 1.0))
        h0 = area2 / L
        scale_u = max(h0, d, 1e-6 * L) / L
        bu = sorted(set([u0 - x for x in graded_intervals(u0, scale_u) if u0 - x >= 0.0] +
                        [u0 + x for x in graded_intervals(1.0 - u0, scale_u) if u0 + x <= 1.0]))
        for u_0, u_1 in zip(bu[:-1], bu[1:]):
            if u_1 - u_0 <= 0.0:
                continue
            ug, uw = gauss_legendre(order, u_0, u_1)
            for s0, s1 in zip(br[:-1], br[1:]):
                sg, sw = gauss_legendre(order, s0, s1)
                S, U = np.meshgrid(sg, ug, indexing="ij")
                W = np.outer(sw, uw) * S * area2 * sgn
                pts = p + S[..., None] * ((1 - U)[..., None] * (a - p) + U[..., None] * (b - p))
                vals = fun(pts.reshape(-1, 3))
                vals = vals.reshape(W.shape + vals.shape[1:])
                total = total + np.tensordot(W, vals, axes=([0, 1], [0, 1]))
    return total
