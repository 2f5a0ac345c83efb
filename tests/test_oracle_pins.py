"""Pins of the CPU oracle to facts outside itself (quadrature exactness, closed forms vs brute
force, Mie series published values and limits, topology invariants, BC defining properties).

A plausible slip anywhere in the oracle (a dropped term, a flipped sign, a transposed index)
fails one of these.
"""
from __future__ import annotations

import math
from pathlib import Path

import numpy as np
import pytest

import meshgen
from oracle import mesh as M
from oracle import mie
from oracle import operators as O
from oracle import potentials as P
from oracle import quadrature as Q

GOLDEN = Path(__file__).resolve().parent / "golden"


# ------------------------------------------------------------------ quadrature

def _monomial_exact(a, b):
    # int over the reference triangle (0,0),(1,0),(0,1) of x^a y^b = a! b! / (a+b+2)!
    return math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)


@pytest.mark.parametrize("rule,degree", [(Q.q7, 5), (Q.q3, 2)])
def test_rule_exact_to_its_degree(rule, degree):
    bary, w = rule()
    assert abs(w.sum() - 1.0) < 1e-15
    x, y = bary[:, 1], bary[:, 2]
    worst_in, worst_out = 0.0, 0.0
    for a in range(degree + 2):
        for b in range(degree + 2 - a):
            approx = 0.5 * np.sum(w * x ** a * y ** b)
            err = abs(approx - _monomial_exact(a, b)) / _monomial_exact(a, b)
            if a + b <= degree:
                worst_in = max(worst_in, err)
            else:
                worst_out = max(worst_out, err)
    assert worst_in < 1e-14
    assert worst_out > 1e-6  # and not beyond: it is the rule it claims to be


def test_subdivided_rule_integrates_smooth_function():
    pts, w = Q.subdivided(Q.q7(), 3)
    f = lambda x, y: np.exp(x) * np.cos(y)
    # reference by Gauss-Legendre in collapsed coordinates (library primitive)
    u, wu = Q.gauss_legendre(40)
    U, V = np.meshgrid(u, u, indexing="ij")
    X, Y = U, V * (1 - U)
    exact = np.sum(np.outer(wu, wu) * (1 - U) * f(X, Y))
    approx = 0.5 * np.sum(w * f(pts[:, 1], pts[:, 2]))
    assert abs(approx - exact) < 1e-9


# ----------------------------------------------------- closed-form potentials

TRI = np.array([[0.0, 0.0, 0.0], [1.2, 0.1, 0.05], [0.3, 0.9, -0.1]])
OBS = [np.array([0.4, 0.3, 0.5]), np.array([0.4, 0.3, 0.02]), np.array([2.0, 1.0, 0.3]),
       TRI.mean(0) + np.array([0, 0, 1e-3]), np.array([-0.5, -0.2, 0.0]),
       0.5 * (TRI[0] + TRI[1]) + np.array([0.0, 0.0, 0.01]), 0.5 * (TRI[0] + TRI[2]) + np.array([-0.02, 0.01, 0.0])]


def _normal(v):
    n = np.cross(v[1] - v[0], v[2] - v[0])
    return n / np.linalg.norm(n)


@pytest.mark.parametrize("i", range(len(OBS)))
def test_static_potentials_vs_brute_force(i):
    r = OBS[i]
    n = _normal(TRI)
    b1 = Q.brute_inner(lambda p: 1 / np.linalg.norm(p - r, axis=1), r, TRI, 20)
    assert abs(P.int_inv_r(r, TRI) - b1) < 1e-12 * abs(b1)
    bv = Q.brute_inner(lambda p: (p - r) / np.linalg.norm(p - r, axis=1)[:, None], r, TRI, 20)
    got = P.int_rp_minus_r_over_r(r, TRI)
    assert np.abs(got - bv).max() < 1e-12 * np.abs(bv).max()
    d = (r - TRI[0]) @ n
    if abs(d) > 1e-9:
        bj = Q.brute_inner(lambda p: (r - p) / np.linalg.norm(p - r, axis=1)[:, None] ** 3, r, TRI, 20)
        got = P.int_rmr_over_r3(r, TRI)
        assert np.abs(got - bj).max() < 1e-10 * np.abs(bj).max()


def test_solid_angle_limit():
    # just above the interior of a large triangle, the normal part of int (r-r')/R^3 tends to 2 pi
    big = np.array([[-50.0, -50.0, 0.0], [100.0, -50.0, 0.0], [-50.0, 100.0, 0.0]])
    j = P.int_rmr_over_r3(np.array([0.1, 0.2, 1e-9]), big)
    assert abs(j[2] - 2 * math.pi) < 0.05
    j = P.int_rmr_over_r3(np.array([0.1, 0.2, -1e-9]), big)
    assert abs(j[2] + 2 * math.pi) < 0.05


def test_remainder_series_continuity():
    # both branches of the regularised kernels agree at the switch point
    k = 3.0 - 0.4j
    R0 = O.SERIES_KR / abs(k)
    for fn, full in ((O.green_remainder, lambda R: O.green(k, R) - 1 / (4 * math.pi * R)),
                     (O.grad_green_remainder,
                      lambda R: O.grad_green_scalar(k, R) + 1 / (4 * math.pi * R ** 3) + k * k / (8 * math.pi * R))):
        a = fn(k, np.array([R0 * (1 - 1e-12)]))[0]
        b = full(R0 * (1 + 1e-12))
        assert abs(a - b) < 1e-12 * abs(b)
    assert abs(O.grad_green_remainder(k, np.array([0.0]))[0] - 1j * k ** 3 / (12 * math.pi)) < 1e-15


# ------------------------------------------------------------------ Mie series

def test_mie_bhmie_published_example():
    """Bohren & Huffman (1983), appendix A, BHMIE test case: m = 1.55, sphere radius 0.525,
    wavelength 0.6328 -> QEXT = QSCA = 3.10543, QBACK = 2.92534 (printed to 6 digits)."""
    vals = dict(l.split("=") for l in (GOLDEN / "bhmie_example.txt").read_text().split("\n")
                if "=" in l and not l.startswith("#"))
    x = 2 * math.pi * float(vals["radius"]) / float(vals["wavelength"])
    qext, qsca, qback = mie.efficiencies(float(vals["m"]), x)
    assert abs(qext - float(vals["qext"])) < 6e-6
    assert abs(qsca - float(vals["qsca"])) < 6e-6
    assert abs(qback - float(vals["qback"])) < 6e-6


def test_mie_rayleigh_limit():
    a, k, eps = 1.0, 0.01, 4.0
    th = np.array([0.0, math.pi / 3, math.pi / 2])
    s = mie.bistatic_rcs(eps, a, k, th, 0.0)
    ray = 4 * math.pi * k ** 4 * a ** 6 * abs((eps - 1) / (eps + 2)) ** 2 * np.cos(math.pi - th) ** 2
    assert np.allclose(s[[0, 1]], ray[[0, 1]], rtol=1e-3)
    s90 = mie.bistatic_rcs(eps, a, k, th, math.pi / 2)
    assert np.allclose(s90, 4 * math.pi * k ** 4 * a ** 6 * abs((eps - 1) / (eps + 2)) ** 2, rtol=1e-3)


def test_mie_energy_conservation_lossless():
    qe, qs, _ = mie.efficiencies(2.0, 3.0)
    assert abs(qe - qs) < 1e-12 * qe
    qe, qs, _ = mie.efficiencies(np.sqrt(np.conj(2.5 - 0.1j)), 3.0)
    assert qe > qs  # absorption with the e^{+j omega t} loss sign conjugated


# ------------------------------------------------------------ topology and BC

@pytest.fixture(scope="module")
def ico2():
    x, t = meshgen.icosphere(2)
    topo = M.build_topology(x, t)
    return topo, M.buffa_christiansen(topo)


def test_topology_invariants(ico2):
    topo, _ = ico2
    nt, ne, nv = len(topo.tri), len(topo.edges), len(topo.xyz)
    assert nv - ne + nt == 2 and ne == 3 * nt // 2
    D = M.incidence_D(topo)
    assert np.abs(np.asarray(D.sum(axis=0))).max() == 0  # every edge leaves one triangle, enters one
    B, F, _ = M.charge_maps(topo)
    assert np.abs((F @ B).toarray() - np.eye(nt - 1)).max() == 0
    # RWG divergence theorem: flux of f_n out of T+ is +1 and into T- is -1 (checked by D . 1/A)
    assert np.all(np.asarray(D[topo.tplus, np.arange(ne)]).ravel() == 1)


def test_mesh_validation_rejects_bad_meshes():
    x, t = meshgen.icosphere(1)
    with pytest.raises(M.MeshError):
        M.build_topology(x, t[:-1])                     # open
    t2 = t.copy(); t2[0] = t2[0][[0, 2, 1]]
    with pytest.raises(M.MeshError):
        M.build_topology(x, t2)                         # inconsistent orientation
    with pytest.raises(M.MeshError):
        M.build_topology(x, t[:, [0, 2, 1]])            # inward


def _bc_field(bary, n):
    """Per sub-triangle linear form (alpha, beta) of BC function n, from its RWG expansion."""
    idx, alpha, beta = O.bc_on_subtriangles(bary)
    out = {}
    for s in range(len(bary.tri)):
        for b in range(idx.shape[1]):
            if idx[s, b] == n:
                out[s] = (alpha[s, b], beta[s, b])
    return out


def _edge_flux(bary, s, p, q, field):
    """Flux of the field of sub-triangle s out through its edge (p, q) (Gauss-Legendre on the edge)."""
    a, b = bary.xyz[p], bary.xyz[q]
    c = bary.xyz[[v for v in bary.tri[s] if v not in (p, q)][0]]
    t = b - a
    nrm = np.cross(np.cross(b - a, c - a), t)
    nrm = -nrm / np.linalg.norm(nrm)  # outward (away from c)
    if nrm @ (c - a) > 0:
        nrm = -nrm
    al, be = field
    A = bary.area[s]
    u, wu = Q.gauss_legendre(4)
    pts = a[None, :] + u[:, None] * t[None, :]
    g = (al * pts - be[None, :]) / (2 * A)
    return np.linalg.norm(t) * np.sum(wu * (g @ nrm))


@pytest.mark.parametrize("n", [0, 37, 111, 479])
def test_bc_defining_fluxes(ico2, n):
    topo, bary = ico2
    va, vb = topo.edges[n]
    assert bary.vs[n] == va and bary.vt[n] == vb  # orientation reading: g_n ~ n x f_n flows va -> vb
    fields = _bc_field(bary, n)
    val = M.valence(topo)
    # support: the dual cells of both end vertices, 2(N_s + N_t) sub-triangles
    assert len(fields) == 2 * (val[va] + val[vb])
    assert set(bary.corner[list(fields)]) == {va, vb}
    nv, ne = len(topo.xyz), len(topo.edges)
    m = nv + n
    for s, fld in fields.items():
        v0, v1, v2 = bary.tri[s]
        out = {}
        for (p, q) in ((v0, v1), (v1, v2), (v2, v0)):
            out[(min(p, q), max(p, q))] = _edge_flux(bary, s, p, q, fld)
        # net emission 1/(2N) in the source cell, absorption 1/(2N) in the sink cell
        cv = bary.corner[s]
        expect = 1 / (2 * val[cv]) if cv == va else -1 / (2 * val[cv])
        assert abs(sum(out.values()) - expect) < 1e-12
        for (p, q), f in out.items():
            if m in (p, q) and (p >= nv + ne or q >= nv + ne):  # a half of the dual edge of n
                assert abs(abs(f) - 0.5) < 1e-12
                assert (f > 0) == (cv == va)  # from the vs side to the vt side
            elif m in (p, q) and min(p, q) < nv:  # primal half-edge of n
                assert abs(f) < 1e-12
            elif p >= nv and q >= nv:  # outer boundary of the dual cell: no flux
                assert abs(f) < 1e-12
        # normal continuity across interior barycentric edges is checked pairwise below
    for s, fld in fields.items():
        for (p, q) in ((bary.tri[s][0], bary.tri[s][1]), (bary.tri[s][1], bary.tri[s][2]), (bary.tri[s][2], bary.tri[s][0])):
            for s2, fld2 in fields.items():
                if s2 != s and p in bary.tri[s2] and q in bary.tri[s2]:
                    assert abs(_edge_flux(bary, s, p, q, fld) + _edge_flux(bary, s2, p, q, fld2)) < 1e-12


def test_gram_Ix_well_conditioned_under_refinement():
    conds = []
    for level in (1, 2, 3):
        x, t = meshgen.icosphere(level)
        topo = M.build_topology(x, t)
        Ix = O.gram_Ix(topo, M.buffa_christiansen(topo))
        assert np.all(np.diag(Ix) > 0)
        conds.append(np.linalg.cond(Ix))
    assert max(conds) < 10.0 and conds[2] < 1.5 * conds[0]


def test_near_rows_equal_near_pairs():
    xyz, tri = meshgen.cubed_sphere(4, (1.0, 0.6, 0.4))
    topo = M.build_topology(meshgen.jitter(xyz, tri, 0.02, 3), tri)
    full = O.near_pairs(topo)
    rows = np.array([0, 17, 50, len(tri) - 1])
    part = O.near_rows(topo, rows)
    assert np.array_equal(part[rows], full[rows])
    assert not np.delete(part, rows, axis=0).any()
