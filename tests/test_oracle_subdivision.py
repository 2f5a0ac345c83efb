"""Pins of the source-rule subdivision for highly conductive objects: where |Re k| h > 2 the
source integration piece is split 4-to-1 until every piece is at most two skin depths across.
At |Re k| h = 6 (80-triangle sphere, k = 6 (1 - j) / h) the subdivided rules (level 2 for the
primal triangles of L, level 2 for the barycentric sub-triangles of K~) agree with a level-4
(L: level-5) composite reference to 1e-5 (far) and a few 1e-3 (near remainder), while the plain
Q7 / Q3 rules miss by 1e-3 .. 0.2: a dropped or misapplied level shows up here."""
from __future__ import annotations

import numpy as np
import pytest

import meshgen
from oracle import mesh as OM
from oracle import operators as OO
from oracle import quadrature as Q

TESTS = np.array([0, 7, 19, 33, 41, 58, 66, 79])


@pytest.fixture(scope="module")
def sphere():
    xyz, tri = meshgen.icosphere(1)
    topo = OM.build_topology(xyz, tri)
    bary = OM.buffa_christiansen(topo)
    return topo, bary, OO.near_pairs(topo), OO.bc_on_subtriangles(bary)


def test_subdivision_level():
    k = 3.0 - 40.0j   # only Re k counts
    h = np.array([0.5, 2.0 / 3.0 - 1e-12, 2.0 / 3.0 + 1e-12, 1.4, 2.7, 100.0])
    assert OO.subdivision_level(k, h).tolist() == [0, 0, 1, 2, 3, OO.SUBDIV_MAX]
    assert OO.subdivision_level(-3.0 + 0j, 1.0) == 1


def test_L_entries_against_fine_rule(sphere):
    topo, bary, near, _ = sphere
    V = OO.tri_vertices(topo)
    k = 6.0 / OO.longest_edge(V).max() * (1 - 1j)
    assert set(OO.subdivision_level(k, OO.longest_edge(V))) == {2}
    _, Lp1 = OO.fill_L(topo, k, near, test_subset=TESTS)
    _, Lp0 = OO.fill_L(topo, k, near, test_subset=TESTS, subdivide=False)
    bq, wq = Q.q7()
    _, Lpn = OO.fill_L(topo, k, near, inner_rule=Q.subdivided((bq, wq), 5), test_subset=TESTS, subdivide=False)
    Lpf = np.zeros_like(Lp1)
    LAf = np.zeros((len(topo.edges), len(topo.edges)), complex)
    pts = Q.points(V, bq)
    for t in TESTS:
        far_idx = np.nonzero(~near[t])[0]
        OO._fill_L_far(topo, k, t, far_idx, pts[t], wq, Q.subdivided((bq, wq), 5), V,
                       topo.tri_signs[t].astype(np.float64), LAf, Lpf)
    far = ~near[TESTS]
    nr = near[TESTS]
    err = lambda a, b, m: np.abs(a[TESTS][m] - b[TESTS][m]).max() / np.abs(b[TESTS][m]).max()
    e1, e0 = err(Lp1, Lpf, far), err(Lp0, Lpf, far)
    n1, n0 = err(Lp1, Lpn, nr), err(Lp0, Lpn, nr)
    print(f"L^phi far: subdivided {e1:.1e}, plain {e0:.1e}; near: subdivided {n1:.1e}, plain {n0:.1e}")
    assert e1 < 1e-5 and e0 > 1e-3
    assert n1 < 5e-3 and n0 > 0.1


def test_K_entries_against_fine_rule(sphere):
    topo, bary, near, bcd = sphere
    V = OO.tri_vertices(topo)
    SV = bary.xyz[bary.tri]
    hs = OO.longest_edge(SV)
    k = 6.0 / hs.max() * (1 - 1j)
    assert set(OO.subdivision_level(k, hs)) == {2}
    tests = TESTS[:4]
    b3, w3 = Q.q3()
    bq, wq = Q.q7()
    ref = Q.subdivided((b3, w3), 4)
    ne = len(topo.edges)
    Kf1, Kf0, Kfr = (np.zeros((ne, ne), complex) for _ in range(3))
    for t in tests:
        rk = Q.points(V[t], bq)
        fi = topo.tri_signs[t][:, None, None] * (rk[None, :, :] - V[t][:, None, :]) / (2 * topo.area[t])
        sidx = np.nonzero(~near[t][bary.parent])[0]
        OO._fill_K_far(topo, k, t, sidx, rk, wq, fi, Q.subdivided((b3, w3), 2), SV, bary.area, bcd, Kf1)
        OO._fill_K_far(topo, k, t, sidx, rk, wq, fi, (b3, w3), SV, bary.area, bcd, Kf0)
        OO._fill_K_far(topo, k, t, sidx, rk, wq, fi, ref, SV, bary.area, bcd, Kfr)
    K1 = OO.fill_K(topo, bary, k, near, bcd, test_subset=tests)
    K0 = OO.fill_K(topo, bary, k, near, bcd, test_subset=tests, subdivide=False)
    Kn = OO.fill_K(topo, bary, k, near, bcd, inner_rule=ref, test_subset=tests, subdivide=False)
    e1 = np.abs(Kf1 - Kfr).max() / np.abs(Kfr).max()
    e0 = np.abs(Kf0 - Kfr).max() / np.abs(Kfr).max()
    # near parts: the full fill minus its far part
    near_ref = Kn - Kf0
    n1 = np.abs((K1 - Kf1) - near_ref).max() / np.abs(near_ref).max()
    n0 = np.abs((K0 - Kf0) - near_ref).max() / np.abs(near_ref).max()
    print(f"K far: subdivided {e1:.1e}, plain {e0:.1e}; near: subdivided {n1:.1e}, plain {n0:.1e}")
    assert e1 < 1e-3 and e0 > 1e-2
    assert n1 < 5e-3 and n0 > 0.1
