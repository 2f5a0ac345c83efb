"""Serving loop: requests of different meshes, frequencies, materials and excitation counts
submitted together give the same currents as the same requests solved alone.

Every product row and reduction is computed in a fixed order whatever launch it lands in (a
request's own launch or a grouped launch shared with other requests), so the comparison is
made at 1e-12 relative and the measured difference is printed (it is 0 when bit-identical).
"""
from __future__ import annotations

import time

import numpy as np
import pytest

import meshgen
import paper_2106_06184_amd as B

pytestmark = pytest.mark.gpu


def _requests():
    """(name, xyz, tri, k0 (1/m), eps_r, n_exc) of a small mixed stream."""
    out = []
    xyz, tri = meshgen.icosphere(2)
    out.append(("ico320_k1_eps4", xyz, tri, 1.0, 4.0, 1))
    xyz, tri = meshgen.cube(4)
    out.append(("cube192_k2_lossy", xyz, tri, 2.0, 2.5 - 0.1j, 3))
    xyz, tri = meshgen.cubed_sphere(5, (1.0, 0.6, 0.4))
    out.append(("ell300_k1.5_eps6", xyz, tri, 1.5, 6.0, 2))
    xyz, tri = meshgen.icosphere(1)
    out.append(("ico80_k0.5_eps1.5", xyz, tri, 0.5, 1.5, 1))
    xyz, tri = meshgen.icosphere(2, 0.8)
    out.append(("ico320_r0.8_k2_eps3", xyz, tri, 2.0, 3.0, 1))
    return out


def _problem_and_exc(k0, eps, n_exc, seed):
    prob = B.make_problem(meshgen.freq_from_k0(k0), [eps], [1.0], [0.0], precision=B.BEM_MIXED)
    khat, pol = meshgen.plane_wave_draws(n_exc, seed)
    return prob, B.plane_waves(khat, pol)


OPTS = dict(tol=1e-8, restart=60, maxit=3000, max_refine=8)


def test_results_same_alone_and_in_the_mix():
    specs = _requests()
    # alone: one request at a time through bem_solve
    ctx = B.bem_create(0)
    alone = []
    for i, (name, xyz, tri, k0, eps, n_exc) in enumerate(specs):
        mesh = B.bem_mesh_load(ctx, xyz, tri)
        info = B.bem_mesh_info(ctx, mesh)
        prob, exc = _problem_and_exc(k0, eps, n_exc, 100 + i)
        op = B.bem_assemble(ctx, mesh, prob)
        rc, H, E, rho, si = B.bem_solve(ctx, op, exc, B.solve_opts(**OPTS), info["n_edge"], info["n_tri"])
        assert rc == B.BEM_OK, (name, rc)
        alone.append((H.copy(), E.copy(), rho.copy()))
        B.bem_release(ctx, op)
        B.bem_release(ctx, mesh)
    B.bem_destroy(ctx)

    # in the mix: everything submitted at once (the first request twice) to a fresh context
    ctx = B.bem_create(0)
    reqs, tickets = [], []
    order = list(range(len(specs))) + [0]
    for i in order:
        name, xyz, tri, k0, eps, n_exc = specs[i]
        prob, exc = _problem_and_exc(k0, eps, n_exc, 100 + i)
        r = B.Request(xyz, tri, None, prob, exc, B.solve_opts(**OPTS))
        reqs.append((i, r))
        tickets.append(B.bem_submit(ctx, r))
    done = {}
    t_end = time.time() + 120
    while len(done) < len(tickets):
        assert time.time() < t_end, "serving did not finish"
        for t in tickets:
            if t in done:
                continue
            rc, info = B.bem_poll(ctx, t)
            if rc != B.BEM_PENDING:
                done[t] = (rc, info.seconds)
        time.sleep(0.005)
    launches, products = B.bem_serve_stats(ctx)
    print(f"combiner: {launches} grouped launches carried {products} products")
    for (i, r), t in zip(reqs, tickets):
        rc, sec = done[t]
        assert rc == B.BEM_OK, (specs[i][0], rc)
        worst = 0.0
        for got, want in zip((r.H, r.E, r.rho), alone[i]):
            worst = max(worst, float(np.abs(got - want).max() / np.abs(want).max()))
        print(f"{specs[i][0]}: latency {sec:.3f} s, max rel diff vs alone {worst:.1e}")
        assert worst <= 1e-12, (specs[i][0], worst)
    B.bem_destroy(ctx)
