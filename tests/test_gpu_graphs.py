"""Captured Arnoldi step products (HIP graphs): solves whose step products are replayed from a
captured graph give bitwise the currents of the same solves with direct launches (BEM_GRAPH=0),
in float64, mixed precision (a second graph for the relaxed products), BEM_FP32 (float32
entries in float64 arithmetic, then float32 products) and the eAEFIE
formulation, for one and for five plane waves with restarts short enough that the batch is
compacted (a graph per column count).  Every replay sits between eager launches and host
synchronisations of the Krylov loop, and each is checked through the final currents.  A nested
GMRES (host decisions inside the product) is never captured."""
from __future__ import annotations

import os

import numpy as np
import pytest

import meshgen
import paper_2106_06184_amd as B

pytestmark = pytest.mark.gpu


def _solve(level, prec, form, inner, nexc, restart, graphs):
    os.environ["BEM_GRAPH"] = "1" if graphs else "0"
    try:
        w = meshgen.sphere_workload(level, 1.2, 3.0 - 0.2j)
        khat, pol = meshgen.plane_wave_draws(nexc, 51)
        ctx = B.bem_create(0)
        try:
            mesh = B.bem_mesh_load(ctx, w.xyz, w.tri)
            info = B.bem_mesh_info(ctx, mesh)
            op = B.bem_assemble(ctx, mesh, B.make_problem(w.freq_hz, w.eps_r, w.mu_r, w.sigma, precision=prec,
                                                          inner_mode=inner, formulation=form))
            rc, H, E, rho, si = B.bem_solve(ctx, op, B.plane_waves(khat, pol.astype(np.complex128)),
                                            B.solve_opts(tol=1e-9, restart=restart, maxit=3000),
                                            info["n_edge"], info["n_tri"])
        finally:
            B.bem_destroy(ctx)
    finally:
        os.environ.pop("BEM_GRAPH", None)
    assert rc == B.BEM_OK
    return H, E, rho, si


CASES = [
    ("fp64_schur", B.BEM_FP64, B.BEM_FORM_SLDM, B.BEM_INNER_SCHUR, 1, 100),
    ("mixed_direct", B.BEM_MIXED, B.BEM_FORM_SLDM, B.BEM_INNER_DIRECT, 1, 100),
    ("fp64_5waves_restart8", B.BEM_FP64, B.BEM_FORM_SLDM, B.BEM_INNER_SCHUR, 5, 8),
    ("mixed_5waves_restart8", B.BEM_MIXED, B.BEM_FORM_SLDM, B.BEM_INNER_SCHUR, 5, 8),
    ("fp32_5waves_restart8", B.BEM_FP32, B.BEM_FORM_SLDM, B.BEM_INNER_SCHUR, 5, 8),
    ("eaefie", B.BEM_FP64, B.BEM_FORM_EAEFIE, B.BEM_INNER_AUTO, 3, 100),
]


@pytest.mark.parametrize("name,prec,form,inner,nexc,restart", CASES)
def test_graph_replay_is_bitwise_direct(name, prec, form, inner, nexc, restart):
    Hg, Eg, rg, sg = _solve(2, prec, form, inner, nexc, restart, True)
    Hd, Ed, rd, sd = _solve(2, prec, form, inner, nexc, restart, False)
    print(f"{name}: {sg.graph_steps} of {sg.outer_iters} column-steps replayed, {sg.seconds * 1e3:.1f} ms "
          f"against {sd.seconds * 1e3:.1f} ms direct")
    assert sg.graph_steps > 0 and sd.graph_steps == 0
    assert sg.outer_iters == sd.outer_iters
    assert np.array_equal(Hg, Hd) and np.array_equal(Eg, Ed) and np.array_equal(rg, rd)


def test_nested_gmres_is_not_captured():
    H, E, rho, si = _solve(1, B.BEM_FP64, B.BEM_FORM_SLDM, B.BEM_INNER_GMRES, 1, 100, True)
    assert si.graph_steps == 0
