"""Write brute_fixtures.npz: whole Galerkin entries of L^A, L^phi and K~ on three jittered
Platonic meshes, integrated by brute force straight from their definitions (oracle/brute.py:
singularity-cancelling maps of each triangle pair onto the 4-cube and tensor Gauss-Legendre; no
singularity extraction, no closed forms, no rule set Q).  Calls only the oracle package (and the
seeded mesh generator).  The entries pin the oracle's near-pair fill (tests/test_oracle_brute.py).

    python tests/golden/make_brute_fixtures.py [--procs P]

Meshes: tetrahedron, octahedron and icosahedron inscribed in the unit sphere, every vertex moved
by meshgen.jitter(frac = 0.08, seed = 5) so that no two triangles are congruent; wavenumber
k = 2 - 0.3j.  L^A, L^phi at Gauss orders 10 and 14 (the pair of orders shows the brute force's
own convergence); K~ at order 12 on the tetrahedron and octahedron, and order 10 beside it.
About 20 minutes on 8 cores.
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
from oracle import brute as BG  # noqa: E402
from oracle import mesh as OM  # noqa: E402

K_WAVE = 2.0 - 0.3j
JITTER = (0.08, 5)
MESHES = {"tet": meshgen.tetrahedron, "oct": meshgen.octahedron, "ico": lambda: meshgen.icosphere(0)}
L_ORDERS = (10, 14)
K_ORDERS = (10, 12)
K_MESHES = ("tet", "oct")


def mesh_of(name):
    xyz, tri = MESHES[name]()
    return meshgen.jitter(xyz, tri, *JITTER), tri


def _init():
    threadpool_limits(1)


def _L(args):
    name, n = args
    xyz, tri = mesh_of(name)
    topo = OM.build_topology(xyz, tri)
    return ("L", name, n), BG.L_blocks(topo.xyz, topo.tri, topo.tri_signs, topo.tri_edges, len(topo.edges), K_WAVE, n)


def _K(args):
    name, n, rows = args
    xyz, tri = mesh_of(name)
    topo = OM.build_topology(xyz, tri)
    bary = OM.buffa_christiansen(topo)
    bt = bary.topo
    forms = BG.bc_linear_forms(bary.xyz, bary.tri, bt.tri_signs, bt.tri_edges, bary.C)
    K = BG.K_rows(topo.xyz, topo.tri, topo.tri_signs, topo.tri_edges, bary.xyz, bary.tri, bary.parent, forms,
                  len(topo.edges), K_WAVE, n, rows=rows)
    return ("K", name, n), (rows, K[rows])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--procs", type=int, default=os.cpu_count() or 8)
    ap.add_argument("--out", default=str(Path(__file__).resolve().parent / "brute_fixtures.npz"))
    a = ap.parse_args()
    t0 = time.time()
    jobs = [(_L, (name, n)) for name in MESHES for n in L_ORDERS]
    for name in K_MESHES:
        ne = len(OM.build_topology(*mesh_of(name)).edges)
        for n in K_ORDERS:
            jobs += [(_K, (name, n, [m])) for m in range(ne)]
    out = {}
    with mp.get_context("fork").Pool(a.procs, initializer=_init) as pool:
        res = [pool.apply_async(f, (x,)) for f, x in jobs]
        for r in res:
            key, val = r.get()
            if key[0] == "L":
                out[f"LA_{key[1]}_{key[2]}"], out[f"Lp_{key[1]}_{key[2]}"] = val
            else:
                name = f"K_{key[1]}_{key[2]}"
                if name not in out:
                    ne = val[1].shape[1]
                    out[name] = np.zeros((ne, ne), complex)
                out[name][val[0]] = val[1]
            print(f"{key} done at {time.time() - t0:.0f} s", flush=True)
    np.savez_compressed(a.out, k=K_WAVE, jitter=np.array(JITTER), **out)
    print(f"wrote {a.out} after {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
