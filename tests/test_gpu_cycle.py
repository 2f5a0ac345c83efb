"""Automatic restart cycles that are too short for a hard request.  The automatic cycle keeps the
batch's Krylov basis under 8 GB, so a large request with many plane waves gets short cycles; on an
electrically large object restarted GMRES can stall on them.  The serving mix (seed 5) holds such
a request: a 14700-triangle ellipsoid at k0 a = 9.35, eps_r = 1.63, 53 plane waves (58816
unknowns, 159-step cycles).  With those cycles alone it ends at a residual of 1e-3 after the
3000-step limit; after a sweep runs out of steps the solver lengthens the cycle (here to 1000
steps) and the next sweep converges.  Checked: convergence to 1e-6 with one lengthening, and
eight of the plane waves solved alone with a fixed 1000-step cycle (no lengthening) agree with
their batched columns to the accuracy the residuals allow.  The oracle cannot solve a system of
this size."""
from __future__ import annotations

import numpy as np
import pytest

import meshgen
import paper_2106_06184_amd as B
from tests.bemutil import rel

pytestmark = pytest.mark.gpu

NAME = "ellipsoid14700_k0a9.35_eps1.63_x53"


def test_short_automatic_cycle_is_lengthened():
    stream = meshgen.mixed_stream(64, rate_hz=2.0, seed=5)
    w = [w for _, w in stream if w.name == NAME][0]
    print(f"{w.name}: {len(w.tri)} triangles, {len(w.khat)} plane waves", flush=True)
    ctx = B.bem_create(0)
    try:
        mesh = B.bem_mesh_load(ctx, w.xyz, w.tri, w.obj)
        info = B.bem_mesh_info(ctx, mesh)
        ne, nt = info["n_edge"], info["n_tri"]
        op = B.bem_assemble(ctx, mesh, B.make_problem(w.freq_hz, w.eps_r, w.mu_r, w.sigma, precision=B.BEM_FP32))
        rc, H, E, rho, si = B.bem_solve(ctx, op, B.plane_waves(w.khat, w.pol),
                                        B.solve_opts(tol=1e-6, restart=0, maxit=3000, max_refine=8), ne, nt)
        print(f"automatic cycle: rc {rc}, {si.outer_iters} column-steps, {si.cycle_growths} lengthening(s), "
              f"residual {si.rel_residual:.2e}, {si.seconds:.1f} s", flush=True)
        assert rc == B.BEM_OK
        assert si.cycle_growths == 1
        assert si.rel_residual <= 1e-6
        k = 8
        rc1, H1, E1, rho1, s1 = B.bem_solve(ctx, op, B.plane_waves(w.khat[:k], w.pol[:k]),
                                            B.solve_opts(tol=1e-6, restart=1000, maxit=3000, max_refine=8), ne, nt)
        print(f"fixed 1000-step cycle, {k} waves: rc {rc1}, {s1.outer_iters} column-steps, "
              f"{s1.cycle_growths} lengthening(s), residual {s1.rel_residual:.2e}", flush=True)
        assert rc1 == B.BEM_OK and s1.cycle_growths == 0
        errs = [rel(got, want) for got, want in ((H[:, :k], H1), (E[:, :k], E1), (rho[:, :k], rho1))]
        print(f"batched against alone: H {errs[0]:.2e}, E {errs[1]:.2e}, rho {errs[2]:.2e}", flush=True)
        assert max(errs) < 1e-3, errs
    finally:
        B.bem_destroy(ctx)
