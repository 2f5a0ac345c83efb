"""Near field of a solution: E and H at points outside the objects (oracle; test
infrastructure only).

Sec. II-C, eqs. diffsources / diffsourcesdis: after the equivalence step the object is
replaced by background material and a pair of differential sources on S, the current
J_Delta = (n x H) - (n x H_eq) and the charge rho_Delta = rho - rho_eq, keeps the field in the
exterior region unchanged.  So at any exterior point the scattered field is the field those
two sources radiate in the homogeneous background (wavenumber k_l, eps = eps0 eps_l,
mu = mu0 mu_l) - the paper evaluates such fields along a probe line (Sec. IV-D).  The paper
prints no formula for this step; the reading taken is the standard mixed-potential form of
the field of a surface current and charge in a homogeneous medium (e^{+j omega t}):

    A(r)   = int_S G(r, r') J_Delta(r') dS'
    Phi(r) = (1/eps) int_S G(r, r') rho_Delta(r') dS'
    E(r)   = -j omega mu A(r) - grad Phi(r),      H(r) = curl A(r)

with G = e^{-jkR}/(4 pi R) (eq. hgf).  J_Delta uses the RWG coefficients (a - a_eq)/(j k0)
and rho_Delta the pulse coefficients B (q - q_eq)/c0 of the solved systems.

Per triangle t (area A_t, free vertices v_i, signs s_i, coefficients J_i of its three edges)
J_Delta = (C r' - P)/(2 A_t) with C = sum_i s_i J_i and P = sum_i s_i J_i v_i, and its
charge density is rho_t / A_t (area-normalised pulses).  With the three moments
    I0 = int_t G dS',   I1 = int_t G (r' - r) dS',   Ig = int_t grad_r G dS'
and W = C r - P the triangle contributes
    A += (C I1 + W I0) / (2 A_t),   grad Phi += (rho_t / (eps A_t)) Ig,
    H += Ig x W / (2 A_t)
(the last because (r - r') x (C r' - P) = (r - r') x W).

Quadrature (reading; the paper names no rule for this step): the 7-point rule on each of the
4^L pieces of the triangle, L from |Re k| and the longest edge as in the fill; for a point
closer to the centroid than twice the longest edge the static parts 1/(4 pi R),
(r' - r)/(4 pi R) and -(r - r')/(4 pi R^3) - k^2 (r - r')/(8 pi R) are integrated in closed
form and only the bounded remainders by the rule, on at least the 16 pieces of level
NEAR_LEVEL (the remainders still have a cone-shaped kink under the point, which the plain
7-point rule resolves to only ~1e-3).  The points must lie off the surface.
"""
from __future__ import annotations

import math

import numpy as np

from . import constants as C
from . import operators as O
from . import potentials as PT
from . import quadrature as Q

NEAR_LEVEL = 2   # least subdivision level of the remainder rule on near triangles


def triangle_moments(k, r, V, level=None, near=None):
    """I0 (nt,), I1 (nt, 3), Ig (nt, 3) of the triangles V (nt, 3, 3) at the point r (3,).

    level: subdivision level per triangle (default from k and the longest edge);
    near: boolean per triangle selecting the singularity-extracted form (default: centroid
    closer than NEAR_FACTOR longest edges, and then at least NEAR_LEVEL).  Given explicitly,
    both are used as they are."""
    V = np.asarray(V, dtype=np.float64)
    r = np.asarray(r, dtype=np.float64)
    nt = len(V)
    h = O.longest_edge(V)
    area = 0.5 * np.linalg.norm(np.cross(V[:, 1] - V[:, 0], V[:, 2] - V[:, 0]), axis=1)
    if level is None:
        level = O.subdivision_level(k, h)
    if near is None:
        near = np.linalg.norm(V.mean(axis=1) - r, axis=1) < O.NEAR_FACTOR * h
        level = np.where(near, np.maximum(level, NEAR_LEVEL), level)
    I0 = np.zeros(nt, complex)
    I1 = np.zeros((nt, 3), complex)
    Ig = np.zeros((nt, 3), complex)
    for lev in np.unique(level):
        bq, wq = Q.subdivided(Q.q7(), int(lev))
        for is_near in (False, True):
            sel = np.nonzero((level == lev) & (near == is_near))[0]
            if len(sel) == 0:
                continue
            x = Q.points(V[sel], bq)                       # (m, nq, 3)
            d = x - r                                      # r' - r
            R = np.linalg.norm(d, axis=2)
            if not is_near:
                g = O.green(k, R)
                gg = O.grad_green_scalar(k, R)
                I0[sel] = area[sel] * (g @ wq)
                I1[sel] = area[sel, None] * np.einsum("mq,mqc,q->mc", g, d, wq)
                Ig[sel] = area[sel, None] * np.einsum("mq,mqc,q->mc", gg, -d, wq)
                continue
            g = O.green_remainder(k, R)
            gg = O.grad_green_remainder(k, R)
            i0 = area[sel] * (g @ wq)
            i1 = area[sel, None] * np.einsum("mq,mqc,q->mc", g, d, wq)
            ig = area[sel, None] * np.einsum("mq,mqc,q->mc", gg, -d, wq)
            rr = np.broadcast_to(r, (len(sel), 3))
            s_inv = PT.int_inv_r(rr, V[sel])                  # int 1/R
            s_vec = PT.int_rp_minus_r_over_r(rr, V[sel])      # int (r' - r)/R
            s_j3 = PT.int_rmr_over_r3(rr, V[sel])             # int (r - r')/R^3
            I0[sel] = i0 + s_inv / (4 * math.pi)
            I1[sel] = i1 + s_vec / (4 * math.pi)
            # grad G = [g_rem - 1/(4 pi R^3) - k^2/(8 pi R)] (r - r')
            Ig[sel] = ig - s_j3 / (4 * math.pi) + (k * k / (8 * math.pi)) * s_vec
    return I0, I1, Ig


def differential_sources(ops, sol):
    """J_Delta (RWG coefficients) and rho_Delta (area-normalised pulse coefficients), eq.
    diffsourcesdis."""
    jd = (sol.a - sol.a_eq) / (1j * ops.k0)
    rd = ops.B @ (sol.q - sol.q_eq) / C.C0
    return jd, rd


def radiated_field(ops, jdelta, rhodelta, points):
    """E, H (npts, 3) radiated in the background by J_Delta and rho_Delta."""
    topo = ops.topo
    V = O.tri_vertices(topo)
    area = topo.area
    k = ops.k_bg
    eps = C.EPS0 * ops.eps_bg
    jwmu = 1j * ops.k0 * C.C0 * C.MU0 * ops.mu_bg
    coef = topo.tri_signs * jdelta[topo.tri_edges]             # (nt, 3) s_i J_i
    Csum = coef.sum(axis=1)                                     # C
    P = np.einsum("ti,tic->tc", coef, V)                        # P
    pts = np.atleast_2d(np.asarray(points, dtype=np.float64))
    E = np.zeros((len(pts), 3), complex)
    H = np.zeros((len(pts), 3), complex)
    for p, r in enumerate(pts):
        I0, I1, Ig = triangle_moments(k, r, V)
        W = Csum[:, None] * r[None, :] - P
        A = np.sum((Csum[:, None] * I1 + W * I0[:, None]) / (2 * area[:, None]), axis=0)
        gphi = np.sum((rhodelta / area)[:, None] * Ig, axis=0) / eps
        E[p] = -jwmu * A - gphi
        H[p] = np.sum(np.cross(Ig, W) / (2 * area[:, None]), axis=0)
    return E, H


def near_field(ops, sol, points):
    """Scattered E, H (npts, 3) of a solution at exterior points."""
    jd, rd = differential_sources(ops, sol)
    return radiated_field(ops, jd, rd, points)


def incident_plane_wave(ops, khat, pol, points, E0=1.0):
    """E_inc = E0 pol e^{-j k_l khat . r}, H_inc = khat x E_inc / eta_l (npts, 3)."""
    pts = np.atleast_2d(np.asarray(points, dtype=np.float64))
    khat = np.asarray(khat, dtype=np.float64)
    pol = np.asarray(pol, dtype=np.complex128)
    eta_l = C.ETA0 * np.sqrt(ops.mu_bg / ops.eps_bg)
    ph = np.exp(-1j * ops.k_bg * (pts @ khat))
    E = E0 * ph[:, None] * pol[None, :]
    H = np.cross(np.broadcast_to(khat, E.shape), E) / eta_l
    return E, H
