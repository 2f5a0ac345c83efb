"""Mesh topology, RWG/pulse data, D/F/B and Buffa-Christiansen functions (oracle).

Readings of the paper (Sec. II-B, discretisation of eq. AEFIEint):
  * RWG functions are "area-normalised": f_n = (r - p+)/(2 A+) on T+ and
    (p- - r)/(2 A-) on T-, i.e. unit flux through edge n from T+ into T-, so
    that div f_n = +1/A+ on T+ and -1/A- on T-.
  * Pulses are area-normalised: 1/A_i on T_i.  Hence div f_n = sum_i D_in p_i with
    D the signed triangle/edge incidence matrix (D[T+,n] = +1, D[T-,n] = -1),
    matching the statement that D is an incidence matrix.
  * Edge n = {va < vb}; T+ is the triangle that traverses va -> vb in its
    counter-clockwise vertex order.
  * Charge neutrality (F, B defined in a reference not reproduced): one charge
    per object is eliminated, the object's highest-index triangle.  B maps the
    kept charges to all charges (the removed one is minus their sum), F keeps the
    rows of the kept triangles; F B = I.
  * Barycentric refinement: every triangle (v0, v1, v2) with centroid c and edge
    midpoints m01, m12, m20 splits into (v0,m01,c), (m01,v1,c), (v1,m12,c),
    (m12,v2,c), (v2,m20,c), (m20,v0,c), inheriting orientation.
  * Buffa-Christiansen function g_n (definition in a reference not
    reproduced) is built as a combination of unit-flux barycentric RWGs whose
    coefficients are the fluxes of the standard combinatorial pattern: flux 1/2
    through each half of the dual edge crossing edge n, from the dual cell C(vs)
    into C(vt); zero flux through the primal half-edges of n and through the rest
    of the support boundary; every sub-triangle of C(vs) emits 1/(2 N_vs) and every
    sub-triangle of C(vt) absorbs 1/(2 N_vt) (N_v = number of triangles at v).
    vt is chosen so that g_n points along n x f_n, i.e. (vt - vs) . (n+ x u) > 0
    with u pointing from T+ into T- across the edge.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp


class MeshError(ValueError):
    pass


@dataclass
class Topology:
    xyz: np.ndarray          # (NV, 3)
    tri: np.ndarray          # (NT, 3)
    obj: np.ndarray          # (NT,) object id per triangle
    n_obj: int
    area: np.ndarray         # (NT,)
    normal: np.ndarray       # (NT, 3) unit outward normals
    centroid: np.ndarray     # (NT, 3)
    edges: np.ndarray        # (NE, 2) vertex pairs va < vb
    tplus: np.ndarray        # (NE,)
    tminus: np.ndarray       # (NE,)
    pplus: np.ndarray        # (NE,) free vertex of T+
    pminus: np.ndarray       # (NE,) free vertex of T-
    tri_edges: np.ndarray    # (NT, 3): edge opposite local vertex i of each triangle
    tri_signs: np.ndarray    # (NT, 3): +1 if the triangle is T+ of that edge, else -1
    edge_obj: np.ndarray     # (NE,)


def build_topology(xyz, tri, obj=None) -> Topology:
    xyz = np.asarray(xyz, dtype=np.float64)
    tri = np.asarray(tri, dtype=np.int64)
    nt = len(tri)
    if obj is None:
        obj = np.zeros(nt, dtype=np.int64)
    obj = np.asarray(obj, dtype=np.int64)
    if tri.ndim != 2 or tri.shape[1] != 3 or nt == 0:
        raise MeshError("triangles must be a non-empty (NT, 3) array")
    if tri.min() < 0 or tri.max() >= len(xyz):
        raise MeshError("triangle vertex index out of range")
    if np.any(tri[:, 0] == tri[:, 1]) or np.any(tri[:, 1] == tri[:, 2]) or np.any(tri[:, 0] == tri[:, 2]):
        raise MeshError("triangle with repeated vertex")
    a, b, c = xyz[tri[:, 0]], xyz[tri[:, 1]], xyz[tri[:, 2]]
    cr = np.cross(b - a, c - a)
    dbl = np.linalg.norm(cr, axis=1)
    h = np.max(np.stack([np.linalg.norm(b - a, axis=1), np.linalg.norm(c - b, axis=1),
                         np.linalg.norm(a - c, axis=1)]), axis=0)
    if np.any(dbl <= 1e-12 * h * h):
        raise MeshError("degenerate (zero-area) triangle")
    area = 0.5 * dbl
    normal = cr / dbl[:, None]
    centroid = (a + b + c) / 3.0

    # Directed edge occurrences: local edge i of a triangle is opposite local vertex i.
    dir_from = np.concatenate([tri[:, 1], tri[:, 2], tri[:, 0]])
    dir_to = np.concatenate([tri[:, 2], tri[:, 0], tri[:, 1]])
    free = np.concatenate([tri[:, 0], tri[:, 1], tri[:, 2]])
    owner = np.tile(np.arange(nt), 3)
    local = np.repeat(np.arange(3), nt)
    lo = np.minimum(dir_from, dir_to)
    hi = np.maximum(dir_from, dir_to)
    keys, inverse, counts = np.unique(lo * (len(xyz) + 1) + hi, return_inverse=True, return_counts=True)
    if np.any(counts != 2):
        raise MeshError("mesh is not closed and 2-manifold (edge shared by != 2 triangles)")
    ne = len(keys)
    edges = np.stack([keys // (len(xyz) + 1), keys % (len(xyz) + 1)], axis=1)
    forward = dir_from < dir_to  # occurrence traverses va -> vb
    tplus = np.full(ne, -1)
    tminus = np.full(ne, -1)
    pplus = np.full(ne, -1)
    pminus = np.full(ne, -1)
    tri_edges = np.zeros((nt, 3), dtype=np.int64)
    tri_signs = np.zeros((nt, 3), dtype=np.int64)
    for occ in range(3 * nt):
        n = inverse[occ]
        t = owner[occ]
        i = local[occ]
        tri_edges[t, i] = n
        if forward[occ]:
            if tplus[n] != -1:
                raise MeshError("inconsistent triangle orientation")
            tplus[n] = t
            pplus[n] = free[occ]
            tri_signs[t, i] = 1
        else:
            if tminus[n] != -1:
                raise MeshError("inconsistent triangle orientation")
            tminus[n] = t
            pminus[n] = free[occ]
            tri_signs[t, i] = -1
    if np.any(obj[tplus] != obj[tminus]):
        raise MeshError("objects share an edge (junctions are not supported)")
    objects = np.unique(obj)
    if not np.array_equal(objects, np.arange(len(objects))):
        raise MeshError("object ids must be 0..n_obj-1")
    # vertex manifoldness: the triangles around every vertex form a single fan
    _check_vertex_fans(tri, nt, len(xyz))
    # outward orientation: positive enclosed volume per object
    vol = np.einsum("ij,ij->i", a, np.cross(b, c)) / 6.0
    for o in objects:
        if vol[obj == o].sum() <= 0.0:
            raise MeshError(f"object {o} is not oriented outward (non-positive volume)")
    return Topology(xyz, tri, obj, len(objects), area, normal, centroid, edges,
                    tplus, tminus, pplus, pminus, tri_edges, tri_signs, obj[tplus])


def _check_vertex_fans(tri, nt, nv):
    # Each triangle contributes the arc (next -> prev) around its vertex; the arcs
    # around every vertex must link into a single cycle.
    nxt = {}
    for t in range(nt):
        for i in range(3):
            v = tri[t, i]
            key = (v, tri[t, (i + 1) % 3])
            if key in nxt:
                raise MeshError("non-manifold vertex")
            nxt[key] = tri[t, (i + 2) % 3]
    by_vertex: dict[int, dict[int, int]] = {}
    for (v, u), w in nxt.items():
        by_vertex.setdefault(v, {})[u] = w
    for v, arcs in by_vertex.items():
        start = next(iter(arcs))
        cur = start
        seen = 0
        while True:
            cur = arcs.get(cur)
            seen += 1
            if cur is None or seen > len(arcs):
                raise MeshError("non-manifold vertex")
            if cur == start:
                break
        if seen != len(arcs):
            raise MeshError("non-manifold vertex (several fans)")


def incidence_D(topo: Topology) -> sp.csr_matrix:
    """Signed incidence D (NT x NE): div f_n = sum_i D_in / A_i on T_i."""
    ne = len(topo.edges)
    rows = np.concatenate([topo.tplus, topo.tminus])
    cols = np.concatenate([np.arange(ne), np.arange(ne)])
    vals = np.concatenate([np.ones(ne), -np.ones(ne)])
    return sp.csr_matrix((vals, (rows, cols)), shape=(len(topo.tri), ne))


def charge_maps(topo: Topology):
    """(B, F, kept): B is NT x (NT - n_obj), F is (NT - n_obj) x NT, F B = I.

    The eliminated charge of every object is its highest-index triangle.
    """
    nt = len(topo.tri)
    removed = np.array([np.nonzero(topo.obj == o)[0].max() for o in range(topo.n_obj)])
    kept = np.setdiff1d(np.arange(nt), removed)
    col_of = {int(t): j for j, t in enumerate(kept)}
    rows, cols, vals = [], [], []
    for t in kept:
        rows.append(int(t)); cols.append(col_of[int(t)]); vals.append(1.0)
    for o, r in enumerate(removed):
        for t in kept[topo.obj[kept] == o]:
            rows.append(int(r)); cols.append(col_of[int(t)]); vals.append(-1.0)
    B = sp.csr_matrix((vals, (rows, cols)), shape=(nt, len(kept)))
    F = sp.csr_matrix((np.ones(len(kept)), (np.arange(len(kept)), kept)), shape=(len(kept), nt))
    return B, F, kept


# --------------------------------------------------------- barycentric mesh

@dataclass
class Barycentric:
    xyz: np.ndarray        # vertices: primal (NV), edge midpoints (NE), centroids (NT)
    tri: np.ndarray        # (6 NT, 3) sub-triangles; sub-triangle 6T+s lies in primal T
    parent: np.ndarray     # (6 NT,) primal triangle of each sub-triangle
    area: np.ndarray
    topo: Topology         # barycentric mesh topology (edges, T+/T-, free vertices)
    corner: np.ndarray     # (6 NT,) primal vertex of each sub-triangle (its dual cell)
    C: sp.csr_matrix       # (NE_primal, NE_bary) BC coefficients on barycentric RWGs
    vs: np.ndarray         # (NE,) source vertex of each BC
    vt: np.ndarray         # (NE,) sink vertex of each BC


def barycentric_refinement(topo: Topology):
    nv, ne, nt = len(topo.xyz), len(topo.edges), len(topo.tri)
    mid = 0.5 * (topo.xyz[topo.edges[:, 0]] + topo.xyz[topo.edges[:, 1]])
    xyz = np.concatenate([topo.xyz, mid, topo.centroid])
    sub = np.zeros((6 * nt, 3), dtype=np.int64)
    corner = np.zeros(6 * nt, dtype=np.int64)
    edge_index = {}
    for n, (va, vb) in enumerate(topo.edges):
        edge_index[(int(va), int(vb))] = n
        edge_index[(int(vb), int(va))] = n
    for t in range(nt):
        v0, v1, v2 = (int(x) for x in topo.tri[t])
        m01 = nv + edge_index[(v0, v1)]
        m12 = nv + edge_index[(v1, v2)]
        m20 = nv + edge_index[(v2, v0)]
        c = nv + ne + t
        sub[6 * t:6 * t + 6] = [(v0, m01, c), (m01, v1, c), (v1, m12, c),
                                (m12, v2, c), (v2, m20, c), (m20, v0, c)]
        corner[6 * t:6 * t + 6] = [v0, v1, v1, v2, v2, v0]
    parent = np.repeat(np.arange(nt), 6)
    btopo = build_topology(xyz, sub, topo.obj[parent])
    return xyz, sub, parent, corner, btopo


def buffa_christiansen(topo: Topology) -> Barycentric:
    xyz, sub, parent, corner, bt = barycentric_refinement(topo)
    nv, ne = len(topo.xyz), len(topo.edges)
    bedge = {}
    for j, (u, w) in enumerate(bt.edges):
        bedge[(int(u), int(w))] = j
        bedge[(int(w), int(u))] = j

    def bflux_coeff(u, w, t_from, flux):
        """Coefficient on the barycentric RWG of edge (u,w) for `flux` leaving t_from."""
        j = bedge[(u, w)]
        if bt.tplus[j] == t_from:
            return j, flux
        assert bt.tminus[j] == t_from
        return j, -flux

    # sub-triangles around each primal vertex, as a cyclic sequence
    subs_at = {}
    for s in range(len(sub)):
        subs_at.setdefault(int(corner[s]), []).append(s)

    def cycle_from(v, m_vertex):
        """Sub-triangles of C(v) in cyclic order, starting next to the half-edge (v, m).

        Returns the list of sub-triangles t_1..t_2N and of the barycentric edges
        e_1..e_{2N-1} between consecutive ones (as vertex pairs).
        """
        cell = subs_at[v]
        # the sub-triangles of C(v) containing vertex m_vertex: two of them
        start = [s for s in cell if m_vertex in sub[s]]
        assert len(start) == 2
        order = [start[0]]
        edges_between = []
        prev_edge = (v, m_vertex)
        while len(order) < len(cell):
            s = order[-1]
            others = [int(x) for x in sub[s] if x != v and x != prev_edge[1]]
            assert len(others) == 1
            nxt_vertex = others[0]
            e = (v, nxt_vertex)
            cand = [q for q in cell if q != s and nxt_vertex in sub[q]]
            assert len(cand) == 1
            edges_between.append(e)
            order.append(cand[0])
            prev_edge = e
        # the last sub-triangle must close back onto (v, m)
        assert m_vertex in sub[order[-1]]
        return order, edges_between

    rows, cols, vals = [], [], []
    vs_arr = np.zeros(ne, dtype=np.int64)
    vt_arr = np.zeros(ne, dtype=np.int64)
    for n in range(ne):
        va, vb = (int(x) for x in topo.edges[n])
        tp, tm = int(topo.tplus[n]), int(topo.tminus[n])
        m = nv + n
        # orientation: (vt - vs) . (n+ x u) > 0, u from T+ into T- across the edge
        e_dir = topo.xyz[vb] - topo.xyz[va]
        to_edge = topo.xyz[va] - topo.xyz[topo.pplus[n]]
        u = to_edge - e_dir * (to_edge @ e_dir) / (e_dir @ e_dir)
        w = np.cross(topo.normal[tp], u)
        if e_dir @ w > 0:
            vs, vt = va, vb
        else:
            vs, vt = vb, va
        vs_arr[n], vt_arr[n] = vs, vt
        coeff: dict[int, float] = {}

        def add(j, c):
            coeff[j] = coeff.get(j, 0.0) + c

        # dual-edge halves (m, c+) and (m, c-): flux 1/2 from the vs side to the vt side
        for t in (tp, tm):
            cT = nv + ne + t
            s_side = [s for s in range(6 * t, 6 * t + 6) if corner[s] == vs and m in sub[s]]
            assert len(s_side) == 1
            j, c = bflux_coeff(m, cT, s_side[0], 0.5)
            add(j, c)
        # inside the two dual cells
        for v, sign in ((vs, 1.0), (vt, -1.0)):
            order, between = cycle_from(v, m)
            nvv = len(order) // 2
            for i, (p, q) in enumerate(between, start=1):
                flux = sign * (i - nvv) / (2.0 * nvv)  # leaving t_i into t_{i+1}
                j, c = bflux_coeff(p, q, order[i - 1], flux)
                add(j, c)
        for j, c in coeff.items():
            if c != 0.0:
                rows.append(n); cols.append(j); vals.append(c)
    C = sp.csr_matrix((vals, (rows, cols)), shape=(ne, len(bt.edges)))
    return Barycentric(xyz, sub, parent, bt.area, bt, corner, C, vs_arr, vt_arr)


def valence(topo: Topology) -> np.ndarray:
    return np.bincount(topo.tri.ravel(), minlength=len(topo.xyz))
