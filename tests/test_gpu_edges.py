"""Edge cases on the device: a vertex of the largest supported valence (16: the BC cells take
the wide kernel variant), the boundary of the excitation batch (257 excitations: a full batch of
256 and a ragged tail of one), zero excitations and zero-amplitude excitations, empty products,
and invalid arguments that must fail with BEM_E_INVALID instead of reaching a kernel."""
from __future__ import annotations

import numpy as np
import pytest

import meshgen
import paper_2106_06184_amd as B
from oracle import systems as S
from tests.bemutil import edge_perm, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = B.bem_create(0)
    yield c
    B.bem_destroy(c)


def test_valence16_cells_match_oracle(ctx):
    xyz, tri = meshgen.bipyramid(16)
    obj = np.zeros(len(tri), np.int32)
    freq = meshgen.freq_from_k0(1.5)
    ops = S.assemble(xyz, tri, obj, S.Problem(freq, [3.0 - 0.2j], [1.0], [0.0]))
    mesh = B.bem_mesh_load(ctx, xyz, tri, obj)
    op = B.bem_assemble(ctx, mesh, B.make_problem(freq, [3.0 - 0.2j], [1.0], [0.0]))
    va, vb, _, _ = B.bem_edge_table(ctx, mesh)
    perm = edge_perm(va, vb, ops.topo.edges)
    ne, nt = len(ops.topo.edges), len(ops.topo.tri)
    for block, M in ((B.BEM_BLOCK_K_INT, ops.K_int), (B.BEM_BLOCK_K_BG, ops.K_bg), (B.BEM_BLOCK_IX, ops.Ix),
                     (B.BEM_BLOCK_LA_INT, ops.LA_int)):
        G = B.bem_block_export(ctx, op, block, ne, ne)
        err = rel(G, M[np.ix_(perm, perm)])
        print(f"valence 16: block {block} rel {err:.2e}")
        assert err < 1e-12
    khat, pol = meshgen.plane_wave_draws(1, 3)
    ref = S.solve_augmented(ops, S.rhs(ops, khat[0], pol[0]))
    rc, H, E, rho, si = B.bem_solve(ctx, op, B.plane_waves(khat, pol), B.solve_opts(tol=1e-12, restart=100, maxit=2000),
                                    ne, nt)
    assert rc == B.BEM_OK
    for got, want in ((H[:, 0], ref.H(ops.k0)[perm]), (E[:, 0], ref.E()[perm]), (rho[:, 0], ref.rho(ops.B))):
        assert rel(got, want) < 1e-10
    B.bem_release(ctx, op)


def test_batch_boundary_and_degenerate_excitations(ctx):
    """257 plane waves (one batch of 256 and a ragged tail of 1), two of them with zero amplitude:
    every column equals the solve of that column alone (the batches are independent), the zero
    columns are exactly zero."""
    w = meshgen.sphere_workload(1, 1.0, 4.0)
    mesh = B.bem_mesh_load(ctx, w.xyz, w.tri, w.obj)
    info = B.bem_mesh_info(ctx, mesh)
    op = B.bem_assemble(ctx, mesh, B.make_problem(w.freq_hz, w.eps_r, w.mu_r, w.sigma))
    khat, pol = meshgen.plane_wave_draws(257, 77)
    amp = np.ones(257, complex)
    amp[[5, 256]] = 0.0
    exc = B.plane_waves(khat, pol)
    for i in range(257):
        exc[i].amp = B.c64(amp[i].real, amp[i].imag)
    opts = B.solve_opts(tol=1e-11, restart=60, maxit=2000)
    rc, H, E, rho, si = B.bem_solve(ctx, op, exc, opts, info["n_edge"], info["n_tri"])
    assert rc == B.BEM_OK and si.rel_residual <= 1e-11
    assert not H[:, 5].any() and not H[:, 256].any() and not E[:, 256].any()
    for i in (0, 200, 255):
        rc1, H1, E1, rho1, _ = B.bem_solve(ctx, op, B.plane_waves(khat[i:i + 1], pol[i:i + 1]), opts,
                                           info["n_edge"], info["n_tri"])
        assert rc1 == B.BEM_OK
        assert rel(H[:, i], H1[:, 0]) < 1e-9 and rel(E[:, i], E1[:, 0]) < 1e-9
    B.bem_release(ctx, op)


def test_empty_and_invalid_calls(ctx):
    import torch
    w = meshgen.sphere_workload(1, 1.0, 4.0)
    mesh = B.bem_mesh_load(ctx, w.xyz, w.tri, w.obj)
    info = B.bem_mesh_info(ctx, mesh)
    op = B.bem_assemble(ctx, mesh, B.make_problem(w.freq_hz, w.eps_r, w.mu_r, w.sigma))
    x = torch.zeros(info["n_unknowns"], dtype=torch.complex128, device="cuda")
    B.bem_apply(ctx, op, B.BEM_BLOCK_FINAL, x.data_ptr(), x.data_ptr(), 0)       # no columns: a no-op
    with pytest.raises(B.BemError):
        B.bem_apply(ctx, op, 99, x.data_ptr(), x.data_ptr(), 1)                  # unknown block
    with pytest.raises(B.BemError):
        B.bem_apply(ctx, op, B.BEM_BLOCK_K_M, x.data_ptr(), x.data_ptr(), 1)     # eAEFIE-only block
    with pytest.raises(B.BemError):
        B.bem_solve(ctx, op, B.plane_waves(np.zeros((0, 3)), np.zeros((0, 3))), B.solve_opts(), info["n_edge"],
                    info["n_tri"])                                               # no excitation
    with pytest.raises(B.BemError):
        B.bem_solve(ctx, op, B.plane_waves(w.khat, w.pol), B.solve_opts(tol=0.0), info["n_edge"], info["n_tri"])
    with pytest.raises(B.BemError):
        B.bem_assemble(ctx, mesh, B.make_problem(-1.0, w.eps_r, w.mu_r, w.sigma))  # negative frequency
    with pytest.raises(B.BemError):
        B.bem_assemble(ctx, mesh, B.make_problem(w.freq_hz, w.eps_r, w.mu_r, w.sigma, formulation=7))
    B.bem_release(ctx, op)
