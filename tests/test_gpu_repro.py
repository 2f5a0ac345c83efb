"""Bitwise reproducibility: repeated assemblies of one mesh give identical blocks, and repeated
solves identical currents (every kernel reduces in a fixed order; no atomics)."""
from __future__ import annotations

import numpy as np
import pytest

import meshgen
import paper_2106_06184_amd as B

pytestmark = pytest.mark.gpu


def test_repeated_fill_and_solve_are_bitwise_identical():
    xyz, tri = meshgen.cube(4)
    ctx = B.bem_create(0)
    mesh = B.bem_mesh_load(ctx, xyz, tri)
    info = B.bem_mesh_info(ctx, mesh)
    ne, nt = info["n_edge"], info["n_tri"]
    khat, pol = meshgen.plane_wave_draws(3, 9)
    blocks = [(B.BEM_BLOCK_LA_INT, ne), (B.BEM_BLOCK_LPHI_INT, nt), (B.BEM_BLOCK_K_INT, ne),
              (B.BEM_BLOCK_LA_BG, ne), (B.BEM_BLOCK_LPHI_BG, nt), (B.BEM_BLOCK_K_BG, ne)]
    runs = []
    for _ in range(3):
        op = B.bem_assemble(ctx, mesh, B.make_problem(meshgen.freq_from_k0(2.0), [2.5 - 0.1j], [1.0], [0.0],
                                                      precision=B.BEM_MIXED))
        mats = {b: B.bem_block_export(ctx, op, b, n, n) for b, n in blocks}
        rc, H, E, rho, _ = B.bem_solve(ctx, op, B.plane_waves(khat, pol),
                                       B.solve_opts(tol=1e-8, restart=60, maxit=2000, max_refine=8), ne, nt)
        assert rc == B.BEM_OK
        runs.append((mats, H, E, rho))
        B.bem_release(ctx, op)
    for r in runs[1:]:
        for b, _ in blocks:
            diff = int((r[0][b] != runs[0][0][b]).sum())
            assert diff == 0, (b, diff)
        for got, want in zip(r[1:], runs[0][1:]):
            assert np.array_equal(got, want)
    B.bem_destroy(ctx)


@pytest.mark.parametrize("nexc", [5, 20, 40])
def test_repeated_fp32_solves_are_bitwise_identical(nexc):
    """BEM_FP32 solves of 5, 20 and 40 plane waves (float32 entries in float64 arithmetic before
    the relaxation point on the embedding's 16-real-column tile and on 3M tiles of 24 and 48
    complex columns, float32 products after on tiles of 32, 64 and 96 real columns), three times
    on one operator: the first solve's products include
    the launch tuner's trials of every candidate, the later ones its choice; the currents are
    bitwise identical."""
    xyz, tri = meshgen.cube(6)
    ctx = B.bem_create(0)
    mesh = B.bem_mesh_load(ctx, xyz, tri)
    info = B.bem_mesh_info(ctx, mesh)
    ne, nt = info["n_edge"], info["n_tri"]
    khat, pol = meshgen.plane_wave_draws(nexc, 17)
    op = B.bem_assemble(ctx, mesh, B.make_problem(meshgen.freq_from_k0(2.0), [2.5 - 0.1j], [1.0], [0.0],
                                                  precision=B.BEM_FP32))
    runs = []
    for _ in range(3):
        rc, H, E, rho, si = B.bem_solve(ctx, op, B.plane_waves(khat, pol),
                                        B.solve_opts(tol=1e-7, restart=80, maxit=2000, max_refine=8), ne, nt)
        assert rc == B.BEM_OK
        runs.append((H, E, rho))
    for r in runs[1:]:
        for got, want in zip(r, runs[0]):
            assert np.array_equal(got, want)
    B.bem_destroy(ctx)


def test_sphere5120_fill_is_bitwise_reproducible():
    """The -O3 quadrature fill at full size (the 5120-triangle sphere of the solve benchmark,
    k0 a = 5, eps_r = 2.5 - 0.1j): three assemblies give bitwise identical K~ (interior and
    background), L^A and L^phi blocks."""
    w = meshgen.config_c2()
    ctx = B.bem_create(0)
    try:
        mesh = B.bem_mesh_load(ctx, w.xyz, w.tri)
        info = B.bem_mesh_info(ctx, mesh)
        ne, nt = info["n_edge"], info["n_tri"]
        blocks = [(B.BEM_BLOCK_K_INT, ne), (B.BEM_BLOCK_K_BG, ne), (B.BEM_BLOCK_LA_INT, ne),
                  (B.BEM_BLOCK_LPHI_BG, nt)]
        first = None
        for _ in range(3):
            op = B.bem_assemble(ctx, mesh, B.make_problem(w.freq_hz, w.eps_r, w.mu_r, w.sigma))
            mats = [B.bem_block_export(ctx, op, b, n, n) for b, n in blocks]
            B.bem_release(ctx, op)
            if first is None:
                first = mats
                continue
            for (b, _), got, want in zip(blocks, mats, first):
                diff = int((got != want).sum())
                assert diff == 0, (b, diff)
    finally:
        B.bem_destroy(ctx)
