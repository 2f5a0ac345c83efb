"""Galerkin fill of L^(A), L^(phi), K~, I_x and the plane-wave right-hand side (oracle).

Definitions (Sec. II-B, eqs. opLAhgf, opLphihgf, opKhgf, hgf; testing with
n x RWG, gradient moved onto the test function):
  L^A_mn  = int_Tm int_Tn f_m(r) . f_n(r') G_k(R) dS' dS
  L^phi_ij = (A_i A_j)^-1 int_Ti int_Tj G_k(R) dS' dS
  K~_mn   = int f_m(r) . PV int grad_r G_k(R) x g_n(r') dS' dS
            with grad_r G_k = g_k(R) (r - r'), g_k(R) = -(1 + jkR) e^{-jkR} / (4 pi R^3)
  I_x,mn  = int (n x f_m) . g_n dS                     (BC tested with n x RWG)
  b_m     = eta0^-1 int f_m . E_inc dS,  E_inc = pol E0 e^{-j k_l khat . r}
G_k(R) = e^{-jkR}/(4 pi R).  The reading taken for the unstated numerical
integration (rule set Q):
  * far triangle pairs: Q7 x Q7 (L), Q7 on the test triangle x Q3 on every
    barycentric source sub-triangle (K~);
  * a pair (T, T') is near when the triangles share a vertex or their centroid
    distance is below NEAR_FACTOR * max(longest edge of T, longest edge of T');
  * near pairs: outer Q7; the inner integral is the closed-form static part
    (1/R, and for K~ also 1/R^3) plus Q7 (L) or Q3 (K~) on the bounded
    remainder  G - 1/(4 pi R)  and  g_k + 1/(4 pi R^3) + k^2/(8 pi R);
  * K~ vanishes identically when test and source triangles are coplanar (all
    vectors lie in one plane); such near pairs are set to zero exactly.
  * highly conductive objects (Sec. II-B asks for specialised integration there,
    from a reference that is not available): wherever |Re k| h > 2 for a source
    integration domain of longest edge h (primal triangle for L, barycentric
    sub-triangle for K~), its rule (Q7 or Q3, and the remainder rule of a near
    pair) is applied on the domain split 4-to-1 L times, the least L with
    |Re k| h / 2^L <= 2 (at most SUBDIV_MAX); Re k = 1/skin depth for a good
    conductor, so every piece is at most two skin depths across.  The test
    (outer) rule is unchanged.
  * The jump term of K is the +1/2 I_x printed with K~ in eq. AEFIEintdis; the
    gradient acts on the observation point.
"""
from __future__ import annotations

import math

import numpy as np

from . import quadrature as Q
from . import potentials as P
from .constants import ETA0
from .mesh import Topology, Barycentric

NEAR_FACTOR = 2.0 - 2e-9  # a hair below 2: structured meshes never sit exactly on the threshold
SERIES_KR = 0.5  # |kR| below which the remainders use their power series
SUBDIV_KH = 2.0  # largest |Re k| h of a source integration piece
SUBDIV_MAX = 4   # deepest 4-to-1 subdivision (256 pieces)


def subdivision_level(k: complex, h) -> np.ndarray:
    """Least L >= 0 with |Re k| h / 2^L <= SUBDIV_KH, capped at SUBDIV_MAX (elementwise in h)."""
    x = abs(complex(k).real) * np.asarray(h, dtype=np.float64)
    lev = np.zeros(x.shape, dtype=np.int64)
    for _ in range(SUBDIV_MAX):
        lev += x / 2.0 ** lev > SUBDIV_KH
    return lev


# ----------------------------------------------------------- kernel pieces

def green(k, R):
    return np.exp(-1j * k * R) / (4 * math.pi * R)


def green_remainder(k, R):
    """G_k(R) - 1/(4 pi R) = (e^{-jkR} - 1)/(4 pi R), bounded at R = 0."""
    R = np.asarray(R, dtype=np.float64)
    z = -1j * k * R
    out = np.empty(R.shape, dtype=np.complex128)
    small = np.abs(z) < SERIES_KR
    with np.errstate(divide="ignore", invalid="ignore"):
        out[~small] = (np.exp(z[~small]) - 1.0) / (4 * math.pi * R[~small])
    # (e^z - 1)/R = (-jk) sum_{n>=1} z^(n-1)/n!
    zs = z[small]
    term = np.ones(zs.shape, dtype=np.complex128)
    acc = term.copy()
    for n in range(2, 30):
        term = term * zs / n
        acc = acc + term
    out[small] = (-1j * k) * acc / (4 * math.pi)
    return out


def grad_green_scalar(k, R):
    """g_k(R): grad_r G_k = g_k(R) (r - r')."""
    return -(1 + 1j * k * R) * np.exp(-1j * k * R) / (4 * math.pi * R ** 3)


def grad_green_remainder(k, R):
    """g_k(R) + 1/(4 pi R^3) + k^2/(8 pi R): bounded, tends to j k^3/(12 pi) at R = 0.

    Power series: (1/4pi) sum_{n>=3} (-1)^n (n-1)/n! (jk)^n R^(n-3).
    """
    R = np.asarray(R, dtype=np.float64)
    out = np.empty(R.shape, dtype=np.complex128)
    small = np.abs(k * R) < SERIES_KR
    Rb = R[~small]
    out[~small] = grad_green_scalar(k, Rb) + 1 / (4 * math.pi * Rb ** 3) + k * k / (8 * math.pi * Rb)
    Rs = R[small]
    acc = np.zeros(Rs.shape, dtype=np.complex128)
    jk = 1j * k
    for n in range(3, 40):
        acc = acc + ((-1) ** n) * (n - 1) / math.factorial(n) * jk ** n * Rs ** (n - 3)
    out[small] = acc / (4 * math.pi)
    return out


# ------------------------------------------------------------ geometry

def tri_vertices(topo: Topology) -> np.ndarray:
    return topo.xyz[topo.tri]  # (NT, 3, 3)


def longest_edge(v: np.ndarray) -> np.ndarray:
    return np.max(np.stack([np.linalg.norm(v[:, 1] - v[:, 0], axis=1),
                            np.linalg.norm(v[:, 2] - v[:, 1], axis=1),
                            np.linalg.norm(v[:, 0] - v[:, 2], axis=1)]), axis=0)


def near_pairs(topo: Topology, factor: float = NEAR_FACTOR) -> np.ndarray:
    """Boolean NT x NT matrix of near triangle pairs (shared vertex or close centroids)."""
    nt = len(topo.tri)
    v = tri_vertices(topo)
    h = longest_edge(v)
    c = topo.centroid
    dist = np.linalg.norm(c[:, None, :] - c[None, :, :], axis=2)
    near = dist < factor * np.maximum(h[:, None], h[None, :])
    inc = np.zeros((nt, len(topo.xyz)), dtype=np.int32)
    inc[np.repeat(np.arange(nt), 3), topo.tri.ravel()] = 1
    share = (inc @ inc.T) > 0
    return near | share


def near_rows(topo: Topology, rows, factor: float = NEAR_FACTOR) -> np.ndarray:
    """The given rows of near_pairs (other rows False), for meshes whose full pair matrix is not
    needed: shared vertex or centroid distance below factor * max(longest edges)."""
    nt = len(topo.tri)
    h = longest_edge(tri_vertices(topo))
    c = topo.centroid
    out = np.zeros((nt, nt), dtype=bool)
    for t in np.atleast_1d(rows):
        d = np.linalg.norm(c - c[t], axis=1)
        share = np.isin(topo.tri, topo.tri[t]).any(axis=1)
        out[t] = (d < factor * np.maximum(h, h[t])) | share
    return out


def coplanar(topo: Topology, t: int, others: np.ndarray) -> np.ndarray:
    n = topo.normal
    h = longest_edge(tri_vertices(topo))
    par = np.abs(n[others] @ n[t]) > 1.0 - 1e-12
    dist = np.abs((topo.centroid[others] - topo.centroid[t]) @ n[t])
    return par & (dist < 1e-10 * h[t])


# --------------------------------------------------------------- L^A, L^phi

def fill_L(topo: Topology, k: complex, near=None, outer_rule=None, inner_rule=None, test_subset=None,
           subdivide=True):
    """Return (LA, Lphi) at wavenumber k.

    outer_rule / inner_rule override Q7 for the near pairs only (used by the
    convergence pins); far pairs use Q7 x Q7, the source rule subdivided where
    |Re k| h > 2 (subdivide=False turns that off, for the pins).  test_subset restricts the
    rows that are filled to the given test triangles (used to time a bounded sample).
    """
    nt, ne = len(topo.tri), len(topo.edges)
    V = tri_vertices(topo)
    A = topo.area
    bq, wq = Q.q7()
    ob, ow = outer_rule if outer_rule is not None else (bq, wq)
    ib0 = inner_rule if inner_rule is not None else (bq, wq)
    pts = Q.points(V, bq)                          # (NT, 7, 3)
    if near is None:
        near = near_pairs(topo)
    lev = subdivision_level(k, longest_edge(V)) if subdivide else np.zeros(nt, dtype=np.int64)
    far_rules = {L: Q.subdivided((bq, wq), L) for L in np.unique(lev)}
    near_rules = {L: Q.subdivided(ib0, L) for L in np.unique(lev)}
    LA = np.zeros((ne, ne), dtype=np.complex128)
    Lphi = np.zeros((nt, nt), dtype=np.complex128)
    free = V                                       # free vertex of half i = vertex i
    for t in (range(nt) if test_subset is None else test_subset):
        si = topo.tri_signs[t].astype(np.float64)
        for L in far_rules:
            far_idx = np.nonzero(~near[t] & (lev == L))[0]
            if len(far_idx):
                _fill_L_far(topo, k, t, far_idx, pts[t], wq, far_rules[L], free, si, LA, Lphi)
        for L in near_rules:
            near_idx = np.nonzero(near[t] & (lev == L))[0]
            if len(near_idx):
                _fill_L_near(topo, k, t, near_idx, (ob, ow), near_rules[L], V, A, si, LA, Lphi)
    return LA, Lphi


def _fill_L_far(topo, k, t, far_idx, rk, wq, src_rule, free, si, LA, Lphi):
    """Far pairs (t, far_idx): test Q7 (points rk, weights wq) x the source rule src_rule."""
    sb, sw = src_rule
    rl = Q.points(tri_vertices(topo)[far_idx], sb)                   # (F, L, 3)
    R = np.linalg.norm(rk[None, :, None, :] - rl[:, None, :, :], axis=3)  # (F, 7, L)
    W = wq[None, :, None] * sw[None, None, :] * green(k, R)             # (F, 7, L)
    Lphi[t, far_idx] = W.sum(axis=(1, 2))
    X = rk[None, :, :] - free[t][:, None, :]                         # (3i, 7k, 3)
    Y = rl[:, None, :, :] - free[far_idx][:, :, None, :]             # (F, 3j, L, 3)
    dots = np.einsum("ikc,fjlc->fijkl", X, Y)
    blk = 0.25 * np.einsum("fijkl,fkl->fij", dots, W)
    sj = topo.tri_signs[far_idx].astype(np.float64)
    blk = blk * si[None, :, None] * sj[:, None, :]
    rows = np.broadcast_to(topo.tri_edges[t][None, :, None], blk.shape)
    cols = np.broadcast_to(topo.tri_edges[far_idx][:, None, :], blk.shape)
    np.add.at(LA, (rows.ravel(), cols.ravel()), blk.ravel())


def _fill_L_near(topo, k, t, near_idx, outer, inner_rule, V, A, si, LA, Lphi):
    """Near pairs (t, near_idx): singularity extraction on the inner integral - closed-form
    static parts over the whole source triangle plus inner_rule on the bounded remainder."""
    ob, ow = outer
    ib, iw = inner_rule
    rk = Q.points(V[t], ob)                                          # (K, 3)
    vs = V[near_idx]                                                 # (N, 3, 3)
    rr = np.broadcast_to(rk[:, None, :], (len(rk), len(near_idx), 3))
    vv = np.broadcast_to(vs[None], (len(rk), len(near_idx), 3, 3))
    I1 = P.int_inv_r(rr, vv)                                         # (K, N)
    Iv = P.int_rp_minus_r_over_r(rr, vv)                             # (K, N, 3)
    rl = Q.points(vs, ib)                                            # (N, L, 3)
    dd = rl[None, :, :, :] - rk[:, None, None, :]                    # r' - r  (K, N, L, 3)
    R = np.linalg.norm(dd, axis=3)
    Gr = green_remainder(k, R) * iw[None, None, :] * A[near_idx][None, :, None]
    S0 = I1 / (4 * math.pi) + Gr.sum(axis=2)                         # int G dS'          (K, N)
    S1 = Iv / (4 * math.pi) + np.einsum("knl,knlc->knc", Gr, dd)     # int G (r'-r) dS' (K, N, 3)
    Lphi[t, near_idx] = np.einsum("k,kn->n", ow, S0) / A[near_idx]
    # int G (r' - p_j) dS' = S1 + (r - p_j) S0
    inner = S1[:, :, None, :] + (rk[:, None, None, :] - vs[None, :, :, :]) * S0[:, :, None, None]  # (K,N,3j,3)
    X = rk[None, :, :] - V[t][:, None, :]                            # (3i, K, 3)
    blk = np.einsum("k,ikc,knjc->nij", ow, X, inner) / (4 * A[near_idx])[:, None, None]
    sj = topo.tri_signs[near_idx].astype(np.float64)
    blk = blk * si[None, :, None] * sj[:, None, :]
    rows = np.broadcast_to(topo.tri_edges[t][None, :, None], blk.shape)
    cols = np.broadcast_to(topo.tri_edges[near_idx][:, None, :], blk.shape)
    np.add.at(LA, (rows.ravel(), cols.ravel()), blk.ravel())


# ------------------------------------------------------------------- BC data

def bc_on_subtriangles(bary: Barycentric):
    """For every sub-triangle t: the BC functions supported on it and their linear
    form there, g_n(r') = (alpha r' - beta) / (2 A_t), from the barycentric RWG
    expansion b_j|t = s_jt (r' - q_jt) / (2 A_t)."""
    bt = bary.topo
    ns = len(bary.tri)
    Ccsc = bary.C.tocsc()
    lists = []
    for t in range(ns):
        acc: dict[int, list] = {}
        for e in range(3):
            j = bt.tri_edges[t, e]
            s = bt.tri_signs[t, e]
            q = bary.xyz[bary.tri[t, e]]
            for ptr in range(Ccsc.indptr[j], Ccsc.indptr[j + 1]):
                n = Ccsc.indices[ptr]
                c = Ccsc.data[ptr]
                a = acc.setdefault(int(n), [0.0, np.zeros(3)])
                a[0] += c * s
                a[1] = a[1] + c * s * q
        lists.append(acc)
    maxb = max(len(a) for a in lists)
    idx = np.full((ns, maxb), -1, dtype=np.int64)
    alpha = np.zeros((ns, maxb))
    beta = np.zeros((ns, maxb, 3))
    for t, acc in enumerate(lists):
        for slot, (n, (a, b)) in enumerate(sorted(acc.items())):
            idx[t, slot] = n
            alpha[t, slot] = a
            beta[t, slot] = b
    return idx, alpha, beta


def fill_K(topo: Topology, bary: Barycentric, k: complex, near=None, bcdata=None,
           outer_rule=None, inner_rule=None, test_subset=None, subdivide=True):
    """K~ (NE x NE) at wavenumber k, BC sources on the barycentric refinement (source rules
    subdivided where |Re k| h > 2 for a sub-triangle of longest edge h, unless subdivide=False)."""
    nt, ne = len(topo.tri), len(topo.edges)
    V = tri_vertices(topo)
    A = topo.area
    SV = bary.xyz[bary.tri]                           # (NS, 3, 3)
    SA = bary.area
    bq, wq = Q.q7()
    b3, w3 = Q.q3()
    ob, ow = outer_rule if outer_rule is not None else (bq, wq)
    ib0 = inner_rule if inner_rule is not None else (b3, w3)
    if near is None:
        near = near_pairs(topo)
    if bcdata is None:
        bcdata = bc_on_subtriangles(bary)
    idx, alpha, beta = bcdata
    lev = subdivision_level(k, longest_edge(SV)) if subdivide else np.zeros(len(SV), dtype=np.int64)
    far_rules = {L: Q.subdivided((b3, w3), L) for L in np.unique(lev)}
    near_rules = {L: Q.subdivided(ib0, L) for L in np.unique(lev)}
    K = np.zeros((ne, ne), dtype=np.complex128)
    parent = bary.parent
    for t in (range(nt) if test_subset is None else test_subset):
        rk = Q.points(V[t], bq)                                       # (7, 3)
        fi = topo.tri_signs[t][:, None, None] * (rk[None, :, :] - V[t][:, None, :]) / (2 * A[t])  # (3i,7k,3)
        far_sub = ~near[t][parent]
        for L, rule in far_rules.items():
            sidx = np.nonzero(far_sub & (lev == L))[0]
            if len(sidx):
                _fill_K_far(topo, k, t, sidx, rk, wq, fi, rule, SV, SA, bcdata, K)
        # near: extraction of 1/R^3 and 1/R parts of g_k on each sub-triangle
        near_tris = np.nonzero(near[t])[0]
        cop = coplanar(topo, t, near_tris)
        ncp = near_tris[~cop]
        if len(ncp):
            subs_all = (6 * ncp[:, None] + np.arange(6)[None, :]).ravel()
            for L, rule in near_rules.items():
                subs = subs_all[lev[subs_all] == L]
                if len(subs):
                    _fill_K_near(topo, k, t, subs, (ob, ow), rule, V, A, SV, SA, bcdata, K)
    return K


def _fill_K_far(topo, k, t, sidx, rk, wq, fi, src_rule, SV, SA, bcdata, K):
    """Far sub-triangles sidx of test triangle t: test Q7 x the source rule on each."""
    idx, alpha, beta = bcdata
    sb, sw = src_rule
    A = topo.area
    spts = Q.points(SV[sidx], sb)                                     # (S, L, 3)
    # g_n at the inner points: (alpha r' - beta)/(2 A_s), zero in unused slots  (S, B, L, 3)
    valid = idx[sidx] >= 0
    gval = (alpha[sidx][:, :, None, None] * spts[:, None, :, :] - beta[sidx][:, :, None, :]) \
        / (2 * SA[sidx][:, None, None, None])
    gval = gval * valid[:, :, None, None]
    d = rk[None, :, None, :] - spts[:, None, :, :]                    # (S, 7k, L, 3)
    R = np.linalg.norm(d, axis=3)
    gR = grad_green_scalar(k, R)                                      # (S, 7, L)
    W = (wq[None, :, None] * sw[None, None, :]) * A[t] * SA[sidx][:, None, None] * gR
    # f_i(r_k) . [ (r_k - r'_j) x g_n(r'_j) ]
    cr = np.cross(d[:, None, :, :, :], gval[:, :, None, :, :])        # (S, B, 7, L, 3)
    val = np.einsum("ikc,sbkjc,skj->sib", fi, cr, W)                  # (S, 3i, B)
    rows = np.broadcast_to(topo.tri_edges[t][None, :, None], val.shape)
    cols = np.broadcast_to(idx[sidx][:, None, :], val.shape)
    ok = cols >= 0
    np.add.at(K, (rows[ok], cols[ok]), val[ok])


def _fill_K_near(topo, k, t, subs, outer, inner_rule, V, A, SV, SA, bcdata, K):
    """Near, non-coplanar sub-triangles subs of test triangle t: closed-form 1/R^3 and 1/R
    parts of g_k plus inner_rule on the bounded remainder."""
    idx, alpha, beta = bcdata
    ob, ow = outer
    ib, iw = inner_rule
    rko = Q.points(V[t], ob)
    fio = topo.tri_signs[t][:, None, None] * (rko[None, :, :] - V[t][:, None, :]) / (2 * A[t])
    vs = SV[subs]
    rr = np.broadcast_to(rko[:, None, :], (len(rko), len(subs), 3))
    vv = np.broadcast_to(vs[None], (len(rko), len(subs), 3, 3))
    J = P.int_rmr_over_r3(rr, vv)                                     # int (r-r')/R^3  (K,S,3)
    Iv = P.int_rp_minus_r_over_r(rr, vv)                              # int (r'-r)/R    (K,S,3)
    rl = Q.points(vs, ib)                                             # (S, L, 3)
    dd = rko[:, None, None, :] - rl[None, :, :, :]                    # r - r'          (K,S,L,3)
    R = np.linalg.norm(dd, axis=3)
    h = grad_green_remainder(k, R) * iw[None, None, :] * SA[subs][None, :, None]
    # v(r) = int g_k (r - r') dS'
    v = -J / (4 * math.pi) + (k * k / (8 * math.pi)) * Iv + np.einsum("ksl,kslc->ksc", h, dd)
    # g_n on t written as (alpha r' - beta)/(2A_t); (r-r') x g_n(r') = (r-r') x (alpha r - beta)/(2A_t)
    gr = (alpha[subs][:, :, None, None] * rko[None, None, :, :] - beta[subs][:, :, None, :]) \
        / (2 * SA[subs])[:, None, None, None]                         # (S, B, K, 3)
    cr = np.cross(np.transpose(v, (1, 0, 2))[:, None, :, :], gr)      # (S, B, K, 3)
    vals = np.einsum("ikc,sbkc,k->sib", fio, cr, ow) * A[t]
    rows = np.broadcast_to(topo.tri_edges[t][None, :, None], vals.shape)
    cols = np.broadcast_to(idx[subs][:, None, :], vals.shape)
    ok = cols >= 0
    np.add.at(K, (rows[ok], cols[ok]), vals[ok])


def gram_Ix(topo: Topology, bary: Barycentric, bcdata=None):
    """I_x,mn = int (n x f_m) . g_n dS, exact with Q3 on every sub-triangle."""
    ne = len(topo.edges)
    if bcdata is None:
        bcdata = bc_on_subtriangles(bary)
    idx, alpha, beta = bcdata
    SV = bary.xyz[bary.tri]
    SA = bary.area
    b3, w3 = Q.q3()
    Ix = np.zeros((ne, ne))
    for s in range(len(bary.tri)):
        t = bary.parent[s]
        rp = Q.points(SV[s], b3)
        nrm = topo.normal[t]
        for i in range(3):
            f = topo.tri_signs[t, i] * (rp - topo.xyz[topo.tri[t, i]]) / (2 * topo.area[t])
            nxf = np.cross(nrm[None, :], f)
            for b in range(idx.shape[1]):
                n = idx[s, b]
                if n < 0:
                    continue
                g = (alpha[s, b] * rp - beta[s, b]) / (2 * SA[s])
                Ix[topo.tri_edges[t, i], n] += SA[s] * np.sum(w3 * np.einsum("jc,jc->j", nxf, g))
    return Ix


def rhs_plane_wave(topo: Topology, k_l: complex, khat, pol, E0: complex = 1.0):
    """b_m = eta0^-1 int f_m . pol E0 exp(-j k_l khat . r) dS (Q7 per triangle)."""
    ne = len(topo.edges)
    V = tri_vertices(topo)
    bq, wq = Q.q7()
    pts = Q.points(V, bq)                                           # (NT, 7, 3)
    phase = np.exp(-1j * k_l * np.einsum("tkc,c->tk", pts, np.asarray(khat, dtype=np.float64)))
    b = np.zeros(ne, dtype=np.complex128)
    pol = np.asarray(pol, dtype=np.complex128)
    for i in range(3):
        f = topo.tri_signs[:, i][:, None, None] * (pts - V[:, i][:, None, :]) / (2 * topo.area[:, None, None])
        fdotp = np.einsum("tkc,c->tk", f, pol)
        val = topo.area * np.sum(wq[None, :] * fdotp * phase, axis=1) * E0 / ETA0
        np.add.at(b, topo.tri_edges[:, i], val)
    return b
