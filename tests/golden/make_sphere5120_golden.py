"""Write the oracle's solution of the 5120-triangle dielectric sphere (k0 a = 5,
eps_r = 2.5 - 0.1j, one x-polarised plane wave along -z) to sphere5120_oracle.npz.

Calls only the oracle (and the seeded mesh generator): the four dense fills of rule set Q
(L^A, L^phi, K~ at the object and at the background wavenumber), the Gram matrix I_x and the
reduced single-object system solved by LAPACK LU (equal to the augmented system of eqs.
AEFIEintdis, AEFIEeqvdis, AEFIEextdis to rounding; pinned in the oracle tests).  The fills are
split over host processes in 64 fixed chunks of test triangles, summed in chunk order, so the
result does not depend on the process count.

    python tests/golden/make_sphere5120_golden.py [--procs P] [--level L]

Stored: H, E (oracle edge order), rho (triangle order), the oracle's edge vertex pairs, the
frequency and the wall time.  About 10 minutes on 8 cores, 25 GB.
"""
from __future__ import annotations

import argparse
import multiprocessing as mp
import os
import sys
import time
from pathlib import Path

ROOT = Path(__file__).resolve().parents[2]
sys.path.insert(0, str(ROOT))

import numpy as np  # noqa: E402
from threadpoolctl import threadpool_limits  # noqa: E402

import meshgen  # noqa: E402
from oracle import constants as C  # noqa: E402
from oracle import mesh as M  # noqa: E402
from oracle import operators as O  # noqa: E402
from oracle import systems as S  # noqa: E402

_G = {}


def _worker_init():
    threadpool_limits(1)


def _rows_L(args):
    k, subset = args
    g = _G
    LA, Lp = O.fill_L(g["topo"], k, g["near"], test_subset=subset)
    er = np.unique(g["topo"].tri_edges[subset].ravel())
    return er, LA[er], np.asarray(subset), Lp[subset]


def _rows_K(args):
    k, subset = args
    g = _G
    K = O.fill_K(g["topo"], g["bary"], k, g["near"], g["bcdata"], test_subset=subset)
    er = np.unique(g["topo"].tri_edges[subset].ravel())
    return er, K[er]


def _chunks(nt, n):
    return [list(range(i, nt, n)) for i in range(n)]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--procs", type=int, default=os.cpu_count() or 8)
    ap.add_argument("--level", type=int, default=4)
    ap.add_argument("--out", default=str(Path(__file__).resolve().parent / "sphere5120_oracle.npz"))
    a = ap.parse_args()
    t0 = time.time()
    w = meshgen.sphere_workload(a.level, 5.0, 2.5 - 0.1j)
    topo = M.build_topology(w.xyz, w.tri, w.obj)
    bary = M.buffa_christiansen(topo)
    bcdata = O.bc_on_subtriangles(bary)
    near = O.near_pairs(topo)
    _G.update(topo=topo, bary=bary, bcdata=bcdata, near=near)
    nt, ne = len(topo.tri), len(topo.edges)
    prob = S.Problem(w.freq_hz, w.eps_r, w.mu_r, w.sigma)
    k0 = C.k0_of(prob.freq_hz)
    epsc = C.eps_c(prob.eps_r[0], prob.sigma[0], prob.freq_hz)
    k_int = C.wavenumber(k0, epsc, prob.mu_r[0])
    k_bg = C.wavenumber(k0, prob.eps_bg, prob.mu_bg)
    print(f"topology {time.time() - t0:.1f} s: NT {nt} NE {ne}", flush=True)
    chunks = _chunks(nt, 64)
    mats = {}
    ctx = mp.get_context("fork")
    with ctx.Pool(a.procs, initializer=_worker_init) as pool:
        for name, k in (("int", k_int), ("bg", k_bg)):
            LA = np.zeros((ne, ne), complex)
            Lp = np.zeros((nt, nt), complex)
            for er, la, tr, lp in pool.imap(_rows_L, [(k, c) for c in chunks]):
                LA[er] += la
                Lp[tr] += lp
            print(f"L fill ({name}) done at {time.time() - t0:.1f} s", flush=True)
            K = np.zeros((ne, ne), complex)
            for er, kk in pool.imap(_rows_K, [(k, c) for c in chunks]):
                K[er] += kk
            print(f"K fill ({name}) done at {time.time() - t0:.1f} s", flush=True)
            mats[name] = (LA, Lp, K)
    Ix = O.gram_Ix(topo, bary, bcdata)
    D = M.incidence_D(topo).toarray()
    B, F, _ = M.charge_maps(topo)
    B, F = B.toarray(), F.toarray()
    LA_i, Lp_i, K_i = mats["int"]
    LA_b, Lp_b, K_b = mats["bg"]
    ops = S.Operators(topo, bary, D, B, F, Ix, LA_i, Lp_i, K_i, LA_b, Lp_b, K_b, K_b,
                      k0, [k_int], k_bg, [epsc], list(prob.mu_r), complex(prob.eps_bg),
                      float(prob.mu_bg))
    del mats
    b = S.rhs(ops, w.khat[0], w.pol[0])
    print(f"solving the reduced system ({2 * ne + nt - 1} unknowns) at {time.time() - t0:.1f} s", flush=True)
    a_, e_, x3 = S.solve_reduced_single(ops, b)
    H = a_ / (1j * k0)
    E = e_ * C.ETA0
    rho = (B @ x3) / C.C0
    np.savez_compressed(a.out, H=H, E=E, rho=rho, edges=topo.edges.astype(np.int32),
                        freq_hz=w.freq_hz, seconds=time.time() - t0)
    print(f"wrote {a.out} after {time.time() - t0:.1f} s", flush=True)


if __name__ == "__main__":
    main()
