"""Brute-force Galerkin integration over pairs of flat triangles (oracle; test infrastructure only).

Whole operator entries straight from their definitions (eqs. opLAhgf, opLphihgf, opKhgf with the
kernel of eq. hgf), with no singularity extraction, no closed-form potential and no rule set Q:
it pins the oracle's near-pair assembly in operators.py and shares no code with it.

For a pair of triangles (T, T') of one conforming mesh, int_T int_T' F(r, r') dS' dS is mapped
to integrals over the unit 4-cube on which the integrand is smooth for kernels with a |r - r'|^-1
or |r - r'|^-2 singularity, and integrated by tensor Gauss-Legendre (numpy's leggauss).  The
maps are written out here from the parametrisations of the two triangles from a shared vertex P,
r = P + xi e(alpha), e(alpha) = (1 - alpha)(A1 - P) + alpha (A2 - P), dS = 2|T| xi dxi dalpha:

* common vertex P: split xi >= zeta (zeta = xi t) and zeta >= xi (xi = zeta t); then
  |r - r'| = xi |e(alpha) - t f(beta)| with the last factor bounded away from 0, and the Jacobian
  4|T||T'| xi^3 t cancels the singularity;
* common edge PQ: as above with both e and f starting on Q - P; the remaining singular point
  t = 1, alpha = beta = 0 is a corner of the (1 - t, alpha, beta) cube, removed by the Duffy split
  of the cube into the three pyramids of its largest coordinate (Jacobian lambda^2);
* identical triangles: with delta = alpha - beta, e(alpha) - (1 - s) e(beta) =
  s e(beta) + delta (A2 - A1); the 2-D corner (s, delta) = 0 is removed by the Duffy split of
  each sign of delta, and beta runs over an interval of length 1 - |delta|;
* disjoint triangles: collapsed-square Gauss-Legendre on each triangle; a pair closer than its
  size is split 4-to-1 on both sides first (recursively).
"""
from __future__ import annotations

import math

import numpy as np


def gauss01(n: int):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def cube4(n: int):
    x, w = gauss01(n)
    g = np.stack(np.meshgrid(x, x, x, x, indexing="ij"), axis=-1).reshape(-1, 4)
    wg = np.einsum("i,j,k,l->ijkl", w, w, w, w).ravel()
    return g, wg


def _area2(v):
    return np.linalg.norm(np.cross(v[1] - v[0], v[2] - v[0]))


def _shared(Ta, Tb, tol=1e-12):
    """Index pairs (i, j) with Ta[i] == Tb[j]."""
    sc = max(np.abs(Ta).max(), np.abs(Tb).max(), 1.0)
    out = []
    for i in range(3):
        for j in range(3):
            if np.linalg.norm(Ta[i] - Tb[j]) <= tol * sc:
                out.append((i, j))
    return out


def _edge_dir(P, A1, A2, a):
    return (1.0 - a)[:, None] * (A1 - P)[None, :] + a[:, None] * (A2 - P)[None, :]


def _rule_vertex(P, A1, A2, B1, B2, n):
    u, w = cube4(n)
    xi, t, al, be = u.T
    c = _area2(np.array([P, A1, A2])) * _area2(np.array([P, B1, B2]))
    e, f = _edge_dir(P, A1, A2, al), _edge_dir(P, B1, B2, be)
    W = c * xi ** 3 * t * w
    r1 = P + xi[:, None] * e
    rp1 = P + (xi * t)[:, None] * f
    r2 = P + (xi * t)[:, None] * e
    rp2 = P + xi[:, None] * f
    return np.concatenate([r1, r2]), np.concatenate([rp1, rp2]), np.concatenate([W, W])


def _rule_edge(P, Q, R1, R2, n):
    """T = (P, Q, R1), T' = (P, Q, R2)."""
    u, w = cube4(n)
    xi, lam, p, q = u.T
    c = _area2(np.array([P, Q, R1])) * _area2(np.array([P, Q, R2]))
    rs, rps, ws = [], [], []
    for largest in range(3):  # which of (s, alpha, beta) is the largest: it equals lam
        if largest == 0:
            s, al, be = lam, lam * p, lam * q
        elif largest == 1:
            s, al, be = lam * p, lam, lam * q
        else:
            s, al, be = lam * p, lam * q, lam
        t = 1.0 - s
        e, f = _edge_dir(P, Q, R1, al), _edge_dir(P, Q, R2, be)
        W = c * xi ** 3 * t * lam ** 2 * w
        rs += [P + xi[:, None] * e, P + (xi * t)[:, None] * e]
        rps += [P + (xi * t)[:, None] * f, P + xi[:, None] * f]
        ws += [W, W]
    return np.concatenate(rs), np.concatenate(rps), np.concatenate(ws)


def _rule_identical(P, Q, R0, n):
    u, w = cube4(n)
    xi, lam, a, v = u.T
    c = _area2(np.array([P, Q, R0])) ** 2
    rs, rps, ws = [], [], []
    for s_largest in (True, False):
        if s_largest:
            s, d = lam, lam * a
        else:
            s, d = lam * a, lam
        t = 1.0 - s
        for sign in (1, -1):
            if sign > 0:   # delta = alpha - beta = d >= 0, beta in [0, 1 - d]
                be = (1.0 - d) * v
                al = be + d
            else:          # delta = -d, alpha in [0, 1 - d]
                al = (1.0 - d) * v
                be = al + d
            e, f = _edge_dir(P, Q, R0, al), _edge_dir(P, Q, R0, be)
            W = c * xi ** 3 * t * (1.0 - d) * lam * w
            rs += [P + xi[:, None] * e, P + (xi * t)[:, None] * e]
            rps += [P + (xi * t)[:, None] * f, P + xi[:, None] * f]
            ws += [W, W]
    return np.concatenate(rs), np.concatenate(rps), np.concatenate(ws)


def _tri_gauss(T, n):
    x, w = gauss01(n)
    X, Y = np.meshgrid(x, x, indexing="ij")
    X, Y = X.ravel(), Y.ravel()
    W = np.outer(w, w).ravel() * X * _area2(T)
    pts = T[0] + X[:, None] * (T[1] - T[0]) + (X * Y)[:, None] * (T[2] - T[1])
    return pts, W


def _split4(T):
    m01, m12, m20 = (T[0] + T[1]) / 2, (T[1] + T[2]) / 2, (T[2] + T[0]) / 2
    return [np.array([T[0], m01, m20]), np.array([m01, T[1], m12]), np.array([m20, m12, T[2]]),
            np.array([m01, m12, m20])]


SPLIT_GAP = 0.5   # a disjoint pair whose gap is below SPLIT_GAP x its larger radius is split
SPLIT_DEPTH = 3


def _rule_disjoint(Ta, Tb, n, depth=0):
    ca, cb = Ta.mean(0), Tb.mean(0)
    ra = np.linalg.norm(Ta - ca, axis=1).max()
    rb = np.linalg.norm(Tb - cb, axis=1).max()
    gap = np.linalg.norm(ca - cb) - ra - rb
    if gap < SPLIT_GAP * max(ra, rb) and depth < SPLIT_DEPTH:
        # split the larger triangle (both when comparable)
        pa = _split4(Ta) if ra >= 0.7 * rb else [Ta]
        pb = _split4(Tb) if rb >= 0.7 * ra else [Tb]
        parts = [_rule_disjoint(a, b, n, depth + 1) for a in pa for b in pb]
        return tuple(np.concatenate(x) for x in zip(*parts))
    pa, wa = _tri_gauss(Ta, n)
    pb, wb = _tri_gauss(Tb, n)
    r = np.repeat(pa, len(pb), axis=0)
    rp = np.tile(pb, (len(pa), 1))
    return r, rp, np.outer(wa, wb).ravel()


def pair_rule(Ta, Tb, n: int):
    """Points (r in Ta, r' in Tb) and weights of int_Ta int_Tb . dS' dS for triangles of one
    conforming mesh (identical, sharing an edge, a vertex, or disjoint).  n Gauss points per
    dimension; the common-vertex map, whose integrand has its nearest complex singularities
    closer to the cube, takes n + 6."""
    Ta, Tb = np.asarray(Ta, float), np.asarray(Tb, float)
    sh = _shared(Ta, Tb)
    if len(sh) == 3:
        return _rule_identical(Ta[0], Ta[1], Ta[2], n)
    if len(sh) == 2:
        (i0, j0), (i1, j1) = sh
        ia = 3 - i0 - i1
        ib = 3 - j0 - j1
        return _rule_edge(Ta[i0], Ta[i1], Ta[ia], Tb[ib], n)
    if len(sh) == 1:
        (i0, j0), = sh
        a = [Ta[(i0 + 1) % 3], Ta[(i0 + 2) % 3]]
        b = [Tb[(j0 + 1) % 3], Tb[(j0 + 2) % 3]]
        return _rule_vertex(Ta[i0], a[0], a[1], b[0], b[1], n + 6)
    return _rule_disjoint(Ta, Tb, n)


# ------------------------------------------------------------------ kernels and entries

def green(k, R):
    return np.exp(-1j * k * R) / (4 * math.pi * R)


def grad_green_scalar(k, R):
    """grad_r G_k(|r - r'|) = g (r - r'), g = -(1 + jkR) e^{-jkR} / (4 pi R^3)."""
    return -(1 + 1j * k * R) * np.exp(-1j * k * R) / (4 * math.pi * R ** 3)


def rwg_half(T, i, sign, r):
    """Half i of an RWG on triangle T (free vertex T[i]): sign (r - T[i]) / (2|T|)."""
    return sign * (r - T[i]) / _area2(T)


def L_blocks(xyz, tri, signs, tri_edges, ne, k, n):
    """L^A (ne x ne) and L^phi (nt x nt) by brute force: every triangle pair, all nine
    half-RWG products and the scalar integral at once."""
    nt = len(tri)
    V = xyz[tri]
    A2 = np.array([_area2(v) for v in V])
    LA = np.zeros((ne, ne), complex)
    Lp = np.zeros((nt, nt), complex)
    for a in range(nt):
        for b in range(nt):
            r, rp, w = pair_rule(V[a], V[b], n)
            G = w * green(k, np.linalg.norm(r - rp, axis=1))
            Lp[a, b] = G.sum() / (0.25 * A2[a] * A2[b])
            for i in range(3):
                fi = rwg_half(V[a], i, signs[a, i], r)
                for j in range(3):
                    fj = rwg_half(V[b], j, signs[b, j], rp)
                    LA[tri_edges[a, i], tri_edges[b, j]] += np.sum(G * np.einsum("pc,pc->p", fi, fj))
    return LA, Lp


def bc_linear_forms(sub_xyz, sub_tri, sub_signs, sub_tri_edges, C):
    """For every barycentric sub-triangle t and BC function n supported on it: g_n on t as
    (alpha r' - beta) / (2|t|), from g_n = sum_j C[n, j] b_j with the barycentric RWG halves
    b_j|t = s (r' - q)/(2|t|).  Returns dict t -> list of (n, alpha, beta)."""
    Cc = C.tocsc()
    out = {}
    for t in range(len(sub_tri)):
        acc = {}
        for e in range(3):
            j = sub_tri_edges[t, e]
            s = sub_signs[t, e]
            q = sub_xyz[sub_tri[t, e]]
            for p in range(Cc.indptr[j], Cc.indptr[j + 1]):
                nn = int(Cc.indices[p])
                c = Cc.data[p]
                a = acc.setdefault(nn, [0.0, np.zeros(3)])
                a[0] += c * s
                a[1] = a[1] + c * s * q
        out[t] = [(nn, a, b) for nn, (a, b) in sorted(acc.items())]
    return out


def K_rows(xyz, tri, signs, tri_edges, sub_xyz, sub_tri, sub_parent, forms, ne, k, n, rows=None):
    """K~_mn = sum_{T in supp f_m} sum_{t in supp g_n} int_T int_t f_m(r) . [grad_r G_k x g_n(r')]
    for the test edges `rows` (all when None), every column.  T is split into its six
    barycentric sub-triangles so that every pair belongs to one conforming mesh."""
    V = xyz[tri]
    SV = sub_xyz[sub_tri]
    SA2 = np.array([_area2(v) for v in SV])
    rows = range(ne) if rows is None else rows
    want = set(int(m) for m in rows)
    tests = sorted({int(T) for T in range(len(tri)) if want & set(int(e) for e in tri_edges[T])})
    children = {T: np.nonzero(sub_parent == T)[0] for T in tests}
    K = np.zeros((ne, ne), complex)
    for T in tests:
        mi = [(i, int(tri_edges[T, i])) for i in range(3) if int(tri_edges[T, i]) in want]
        for tau in children[T]:
            for t in range(len(sub_tri)):
                if not forms[t]:
                    continue
                r, rp, w = pair_rule(SV[tau], SV[t], n)
                d = r - rp
                gk = grad_green_scalar(k, np.linalg.norm(d, axis=1)) * w
                fi = np.stack([rwg_half(V[T], i, signs[T, i], r) for i, _ in mi])            # (I, P, 3)
                al = np.array([f[1] for f in forms[t]])
                be = np.array([f[2] for f in forms[t]])
                gn = (al[:, None, None] * rp[None] - be[:, None, :]) / SA2[t]                # (B, P, 3)
                cr = np.cross(d[None], gn)                                                    # (B, P, 3)
                val = np.einsum("p,ipc,bpc->ib", gk, fi, cr)
                for a, (_, m) in enumerate(mi):
                    for b, f in enumerate(forms[t]):
                        K[m, f[0]] += val[a, b]
    return K
