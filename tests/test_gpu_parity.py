"""GPU parity: every dense block, every product and the solve against the float64 oracle.

Cases are small enough for the oracle to finish in seconds while spanning many tiles of
the kernels (80 and 320 triangles, lossless and lossy media).  Tolerances: float64 fill and
products within 1e-12 relative (Frobenius) - the two sides evaluate the same quadrature sums
in a different order; float64 solve within 1e-10 relative with GMRES at 1e-13.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

import meshgen
import paper_2106_06184_amd as B
from oracle import systems as S
from tests.bemutil import edge_perm, final_perm, meq_perm, rel

pytestmark = pytest.mark.gpu

CASES = {
    # name: (icosphere level, k0 a, eps_r (object), eps_bg (background))
    "ico80_eps4": (1, 1.0, 4.0, 1.0),
    "ico80_lossy": (1, 2.0, 2.5 - 0.1j, 1.5 - 0.05j),
}


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    assert torch.cuda.is_available()
    return torch


@pytest.fixture(scope="module")
def ctx():
    c = B.bem_create(0)
    yield c
    B.bem_destroy(c)


_cache = {}
_oracle = {}


def case(name, ctx, inner=B.BEM_INNER_GMRES, precond=0, precision=B.BEM_FP64):
    key = (name, inner, precond, precision)
    if key in _cache:
        return _cache[key]
    level, k0a, eps, eps_bg = CASES[name]
    w = meshgen.sphere_workload(level, k0a, eps)
    if name not in _oracle:
        prob = S.Problem(w.freq_hz, w.eps_r, w.mu_r, w.sigma, eps_bg=eps_bg)
        _oracle[name] = S.assemble(w.xyz, w.tri, w.obj, prob)
    ops = _oracle[name]
    mesh = B.bem_mesh_load(ctx, w.xyz, w.tri)
    p = B.make_problem(w.freq_hz, w.eps_r, w.mu_r, w.sigma, eps_bg=eps_bg, precision=precision, inner_mode=inner,
                       precond=precond)
    op = B.bem_assemble(ctx, mesh, p)
    va, vb, _, _ = B.bem_edge_table(ctx, mesh)
    perm = edge_perm(va, vb, ops.topo.edges)
    _cache[key] = (w, ops, mesh, op, perm)
    return _cache[key]


@pytest.mark.parametrize("backend", ["valu", "mfma"])
def test_device_inverse_of_meq(backend, ctx, monkeypatch):
    """The direct nested solve's device inverse times the oracle's M_eq is the identity (both
    the VALU and the matrix-core rank-64 update of the Gauss-Jordan elimination)."""
    monkeypatch.setenv("BEM_DENSE_VALU", "1" if backend == "valu" else "0")
    level, k0a, eps, eps_bg = CASES["ico80_lossy"]
    w = meshgen.sphere_workload(level, k0a, eps)
    if "ico80_lossy" not in _oracle:
        _oracle["ico80_lossy"] = S.assemble(w.xyz, w.tri, w.obj,
                                            S.Problem(w.freq_hz, w.eps_r, w.mu_r, w.sigma, eps_bg=eps_bg))
    ops = _oracle["ico80_lossy"]
    mesh = B.bem_mesh_load(ctx, w.xyz, w.tri)
    op = B.bem_assemble(ctx, mesh, B.make_problem(w.freq_hz, w.eps_r, w.mu_r, w.sigma, eps_bg=eps_bg,
                                                  inner_mode=B.BEM_INNER_DIRECT, precond=0))
    va, vb, _, _ = B.bem_edge_table(ctx, mesh)
    perm = edge_perm(va, vb, ops.topo.edges)
    ne, nt = len(ops.topo.edges), len(ops.topo.tri)
    Meq, _, _ = S.equivalent_matrix_object(ops, 0)
    P = meq_perm(perm, ne, nt - 1)
    Minv = B.bem_block_export(ctx, op, B.BEM_BLOCK_MEQ_INV, len(Meq), len(Meq))
    err = np.abs(Minv @ Meq[np.ix_(P, P)] - np.eye(len(Meq))).max()
    print(f"{backend}: max |M_eq^-1 M_eq - I| = {err:.2e}")
    B.bem_release(ctx, op)
    assert err < 1e-10


def oracle_blocks(ops):
    return {
        B.BEM_BLOCK_LA_INT: ops.LA_int, B.BEM_BLOCK_LPHI_INT: ops.Lphi_int, B.BEM_BLOCK_K_INT: ops.K_int,
        B.BEM_BLOCK_LA_BG: ops.LA_bg, B.BEM_BLOCK_LPHI_BG: ops.Lphi_bg, B.BEM_BLOCK_K_BG: ops.K_bg,
        B.BEM_BLOCK_IX: ops.Ix,
    }


def permute(block, M, perm):
    if block in (B.BEM_BLOCK_LPHI_INT, B.BEM_BLOCK_LPHI_BG):
        return M
    return M[np.ix_(perm, perm)]


@pytest.mark.parametrize("name", list(CASES))
def test_blocks_match_oracle(name, ctx):
    w, ops, mesh, op, perm = case(name, ctx)
    ne, nt = len(ops.topo.edges), len(ops.topo.tri)
    for block, M in oracle_blocks(ops).items():
        n = nt if block in (B.BEM_BLOCK_LPHI_INT, B.BEM_BLOCK_LPHI_BG) else ne
        G = B.bem_block_export(ctx, op, block, n, n)
        ref = permute(block, M, perm)
        err = rel(G, ref)
        emax = np.abs(G - ref).max() / np.abs(ref).max()
        print(f"{name} block {block}: rel {err:.2e} max {emax:.2e}")
        assert err < 1e-12 and emax < 1e-11, (block, err, emax)


@pytest.mark.parametrize("nrhs", [2, 5])
@pytest.mark.parametrize("name", list(CASES))
def test_apply_matches_oracle(name, nrhs, ctx, torch_mod):
    """Every block times nrhs random columns: 2 columns run as grouped GEMVs, 5 as float64
    matrix-core GEMMs (the nested solve of the final system by GMRES, column by column)."""
    torch = torch_mod
    w, ops, mesh, op, perm = case(name, ctx)
    ne, nt = len(ops.topo.edges), len(ops.topo.tri)
    nq = nt - 1
    rng = np.random.default_rng(7)
    B.bem_set_inner_tol(ctx, op, 1e-14)
    blocks = oracle_blocks(ops)
    Meq, _, _ = S.equivalent_matrix_object(ops, 0)
    blocks[B.BEM_BLOCK_MEQ] = Meq
    blocks[B.BEM_BLOCK_FINAL] = S.final_matrix(ops)
    stream = torch.cuda.current_stream().cuda_stream
    for block, M in blocks.items():
        n = M.shape[0]
        if block == B.BEM_BLOCK_FINAL:
            P = final_perm(perm, ne, nq)
            ref_M = M[np.ix_(P, P)]
        elif block == B.BEM_BLOCK_MEQ:
            P = meq_perm(perm, ne, nq)
            ref_M = M[np.ix_(P, P)]
        else:
            ref_M = permute(block, M, perm)
        x = rng.standard_normal((nrhs, n)) + 1j * rng.standard_normal((nrhs, n))
        xd = torch.tensor(x, dtype=torch.complex128, device="cuda")
        yd = torch.zeros_like(xd)
        B.bem_apply(ctx, op, block, xd.data_ptr(), yd.data_ptr(), nrhs, stream)
        torch.cuda.synchronize()
        y = yd.cpu().numpy()
        ref = x @ ref_M.T
        err = rel(y, ref)
        print(f"{name} apply block {block}: rel {err:.2e}")
        tol = 1e-11 if block == B.BEM_BLOCK_FINAL else 1e-12
        assert err < tol, (block, err)


@pytest.mark.parametrize("inner", [B.BEM_INNER_DIRECT, B.BEM_INNER_SCHUR])
@pytest.mark.parametrize("name", list(CASES))
def test_apply_final_direct_modes(name, inner, ctx, torch_mod):
    """The final system with the nested solve done by the augmented inverse or by the charge-
    eliminated S^-1 (float64 GEMM over 5 columns, GEMV for 1) equals the oracle's matrix."""
    torch = torch_mod
    w, ops, mesh, op, perm = case(name, ctx, inner, 0)
    ne, nt = len(ops.topo.edges), len(ops.topo.tri)
    M = S.final_matrix(ops)
    P = final_perm(perm, ne, nt - 1)
    ref_M = M[np.ix_(P, P)]
    rng = np.random.default_rng(11)
    stream = torch.cuda.current_stream().cuda_stream
    for nrhs in (1, 5):
        x = rng.standard_normal((nrhs, len(M))) + 1j * rng.standard_normal((nrhs, len(M)))
        xd = torch.tensor(x, dtype=torch.complex128, device="cuda")
        yd = torch.zeros_like(xd)
        B.bem_apply(ctx, op, B.BEM_BLOCK_FINAL, xd.data_ptr(), yd.data_ptr(), nrhs, stream)
        torch.cuda.synchronize()
        err = rel(yd.cpu().numpy(), x @ ref_M.T)
        print(f"{name} inner {inner} nrhs {nrhs}: rel {err:.2e}")
        assert err < 1e-11, (nrhs, err)


MODES = [(B.BEM_INNER_GMRES, 0), (B.BEM_INNER_GMRES, 1), (B.BEM_INNER_DIRECT, 0), (B.BEM_INNER_DIRECT, 1),
         (B.BEM_INNER_SCHUR, 0), (B.BEM_INNER_SCHUR, 1)]


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("inner,precond", MODES)
def test_solve_fp64_matches_oracle(name, inner, precond, ctx):
    w, ops, mesh, op, perm = case(name, ctx, inner, precond)
    ne, nt = len(ops.topo.edges), len(ops.topo.tri)
    b = S.rhs(ops, w.khat[0], w.pol[0])
    ref = S.solve_augmented(ops, b)
    exc = B.plane_waves(w.khat, w.pol)
    rc, H, E, rho, info = B.bem_solve(ctx, op, exc, B.solve_opts(tol=1e-13, restart=100, maxit=3000,
                                                                  inner_tol=1e-14), ne, nt)
    print(f"{name} inner {inner} precond {precond}: outer {info.outer_iters} inner max {info.inner_iters_max} "
          f"res {info.rel_residual:.2e}")
    assert rc == B.BEM_OK
    H_ref = ref.H(ops.k0)[perm]
    E_ref = ref.E()[perm]
    rho_ref = ref.rho(ops.B)
    for lab, got, want in (("H", H[:, 0], H_ref), ("E", E[:, 0], E_ref), ("rho", rho[:, 0], rho_ref)):
        err = rel(got, want)
        print(f"  {lab}: rel {err:.2e}")
        assert err < 1e-10, (lab, err)


@pytest.mark.parametrize("inner", [B.BEM_INNER_DIRECT, B.BEM_INNER_SCHUR])
@pytest.mark.parametrize("name", list(CASES))
def test_solve_mixed_matches_oracle(name, inner, ctx):
    """float32 products and nested solves, float64 Arnoldi and residual refinement: after
    refinement to a 1e-9 float64 residual the currents are within 1e-6 of the oracle."""
    w, ops, mesh, op, perm = case(name, ctx, inner, 1, B.BEM_MIXED)
    ne, nt = len(ops.topo.edges), len(ops.topo.tri)
    ref = S.solve_augmented(ops, S.rhs(ops, w.khat[0], w.pol[0]))
    rc, H, E, rho, info = B.bem_solve(ctx, op, B.plane_waves(w.khat, w.pol),
                                      B.solve_opts(tol=1e-9, restart=100, maxit=3000, max_refine=8), ne, nt)
    print(f"{name} mixed: outer {info.outer_iters} refine {info.refine_steps} res {info.rel_residual:.2e}")
    assert rc == B.BEM_OK and info.rel_residual <= 1e-9
    for lab, got, want in (("H", H[:, 0], ref.H(ops.k0)[perm]), ("E", E[:, 0], ref.E()[perm]),
                           ("rho", rho[:, 0], ref.rho(ops.B))):
        err = rel(got, want)
        print(f"  {lab}: rel {err:.2e}")
        assert err < 1e-6, (lab, err)


def test_dense_inverse_of_meq(ctx, torch_mod):
    """The direct nested solve: M_eq times its device inverse applied through the final
    operator equals the oracle's exact Y products (checked via BEM_BLOCK_FINAL above); here the
    equivalent-configuration product itself is checked against the oracle matrix."""
    torch = torch_mod
    w, ops, mesh, op, perm = case("ico80_lossy", ctx, B.BEM_INNER_DIRECT, 1)
    ne, nt = len(ops.topo.edges), len(ops.topo.tri)
    Meq, _, _ = S.equivalent_matrix_object(ops, 0)
    P = meq_perm(perm, ne, nt - 1)
    rng = np.random.default_rng(3)
    x = rng.standard_normal(len(Meq)) + 1j * rng.standard_normal(len(Meq))
    xd = torch.tensor(x, dtype=torch.complex128, device="cuda")
    yd = torch.zeros_like(xd)
    B.bem_apply(ctx, op, B.BEM_BLOCK_MEQ, xd.data_ptr(), yd.data_ptr(), 1, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert rel(yd.cpu().numpy(), Meq[np.ix_(P, P)] @ x) < 1e-12


N_EXC = 6


def _multi_reference(ops, n_exc, seed):
    khat, pol = meshgen.plane_wave_draws(n_exc, seed)
    b = np.stack([S.rhs(ops, khat[i], pol[i]) for i in range(n_exc)], axis=1)
    return khat, pol, S.solve_augmented(ops, b)


@pytest.mark.parametrize("precision", [B.BEM_FP64, B.BEM_MIXED])
@pytest.mark.parametrize("name", list(CASES))
def test_solve_many_excitations(name, precision, ctx):
    """Several plane waves (random directions and polarisations) solved in one batch: every
    Krylov step applies the final system to all unconverged columns with matrix-core GEMMs
    (float64, or float32 with float64 refinement).  Each column matches the oracle's direct
    solve: 1e-10 in float64, 1e-6 after refinement."""
    w, ops, mesh, op, perm = case(name, ctx, B.BEM_INNER_SCHUR, 1, precision)
    ne, nt = len(ops.topo.edges), len(ops.topo.tri)
    khat, pol, refs = _multi_reference(ops, N_EXC, 5)
    fp64 = precision == B.BEM_FP64
    opts = B.solve_opts(tol=1e-13 if fp64 else 1e-9, restart=60, maxit=3000, max_refine=8)
    rc, H, E, rho, info = B.bem_solve(ctx, op, B.plane_waves(khat, pol), opts, ne, nt)
    print(f"{name} prec {precision}: outer {info.outer_iters} refine {info.refine_steps} "
          f"products {info.n_products} res {info.rel_residual:.2e}")
    assert rc == B.BEM_OK
    tol = 1e-10 if fp64 else 1e-6
    for c, ref in enumerate(refs):
        for lab, got, want in (("H", H[:, c], ref.H(ops.k0)[perm]), ("E", E[:, c], ref.E()[perm]),
                               ("rho", rho[:, c], ref.rho(ops.B))):
            err = rel(got, want)
            assert err < tol, (c, lab, err)
