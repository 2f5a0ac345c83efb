"""Closed-form static integrals over a flat triangle (oracle; test infrastructure only).

For an observation point r and a flat triangle T' with unit normal n (counter-
clockwise vertices), write d = n.(r - v0) for the height of r above the plane
and rho for its projection.  For every edge i (from v_i to v_{i+1}) let s be the
unit tangent, m = s x n the outward in-plane normal, s-/s+ the signed positions
of the edge ends along s relative to the foot of rho on the edge line, t0 the
signed distance from rho to the edge line along m, R0^2 = t0^2 + d^2 and
R-/+ the distances from r to the edge ends.  With
    f_i    = ln((R+ + s+)/(R- + s-))
    beta_i = atan(t0 s+/(R0^2 + |d| R+)) - atan(t0 s-/(R0^2 + |d| R-))
the classical potential-integral results (Wilton et al. 1984; Graglia 1993) are
    int 1/R dS'              = sum_i t0_i f_i - |d| sum_i beta_i
    int (rho' - rho)/R dS'   = 1/2 sum_i m_i [R0_i^2 f_i + s+ R+ - s- R-]
    int (r - r')/R^3 dS'     = -grad_r int 1/R dS' = sum_i m_i f_i + sign(d) n sum_i beta_i
These are pinned against brute-force quadrature in the test-suite.  The log is
evaluated in whichever of its equivalent forms avoids cancellation.
"""
from __future__ import annotations

import numpy as np


def _edge_terms(r, v):
    """r: (..., 3); v: (..., 3, 3) triangle vertices.  Returns per-edge arrays."""
    v0, v1, v2 = v[..., 0, :], v[..., 1, :], v[..., 2, :]
    nrm = np.cross(v1 - v0, v2 - v0)
    nrm = nrm / np.linalg.norm(nrm, axis=-1, keepdims=True)
    d = np.einsum("...j,...j->...", r - v0, nrm)
    rho = r - d[..., None] * nrm
    ends = [(v0, v1), (v1, v2), (v2, v0)]
    out = []
    for a, b in ends:
        e = b - a
        ln = np.linalg.norm(e, axis=-1, keepdims=True)
        s = e / ln
        m = np.cross(s, nrm)
        sm = np.einsum("...j,...j->...", a - rho, s)
        sp_ = np.einsum("...j,...j->...", b - rho, s)
        t0 = np.einsum("...j,...j->...", a - rho, m)
        r02 = t0 * t0 + d * d
        rm = np.sqrt(r02 + sm * sm)
        rp = np.sqrt(r02 + sp_ * sp_)
        with np.errstate(divide="ignore", invalid="ignore"):
            f_pos = np.log((rp + sp_) / (rm + sm))
            f_neg = np.log((rm - sm) / (rp - sp_))
            f_mix = np.log((rp + sp_) * (rm - sm) / r02)
        f = np.where(sm >= 0, f_pos, np.where(sp_ <= 0, f_neg, f_mix))
        ad = np.abs(d)
        beta = np.arctan2(t0 * sp_, r02 + ad * rp) - np.arctan2(t0 * sm, r02 + ad * rm)
        out.append((m, sm, sp_, t0, r02, rm, rp, f, beta))
    return nrm, d, out


def int_inv_r(r, v):
    """int_T' 1/R dS'."""
    _, d, edges = _edge_terms(r, v)
    tot = 0.0
    for (m, sm, sp_, t0, r02, rm, rp, f, beta) in edges:
        tot = tot + np.where(np.abs(t0) > 0, t0 * f, 0.0) - np.abs(d) * beta
    return tot


def int_rho_over_r(r, v):
    """int_T' (rho' - rho)/R dS' (in-plane vector)."""
    _, d, edges = _edge_terms(r, v)
    tot = 0.0
    for (m, sm, sp_, t0, r02, rm, rp, f, beta) in edges:
        term = np.where(r02 > 0, r02 * f, 0.0) + sp_ * rp - sm * rm
        tot = tot + 0.5 * m * term[..., None]
    return tot


def int_rmr_over_r3(r, v):
    """int_T' (r - r')/R^3 dS' (vector), for r not on the triangle's closure."""
    nrm, d, edges = _edge_terms(r, v)
    tot = 0.0
    bsum = 0.0
    for (m, sm, sp_, t0, r02, rm, rp, f, beta) in edges:
        tot = tot + m * f[..., None]
        bsum = bsum + beta
    return tot + (np.sign(d) * bsum)[..., None] * nrm


def int_rp_minus_r_over_r(r, v):
    """int_T' (r' - r)/R dS' = int (rho' - rho)/R dS' - d n int 1/R dS'."""
    nrm, d, _ = _edge_terms(r, v)
    return int_rho_over_r(r, v) - (d * int_inv_r(r, v))[..., None] * nrm
