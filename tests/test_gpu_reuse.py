"""Repeated objects (Sec. II-F): translated copies share their object-local blocks and
inverses.  Every block, the final-system product and the solve still match the oracle, which
fills every object on its own (1e-12 for blocks, 1e-11 for the composed product, 1e-10 for
float64 solves, 1e-6 after mixed-precision refinement), and the shared assembly gives the same
currents as the unshared one."""
from __future__ import annotations

import numpy as np
import pytest

import meshgen
import paper_2106_06184_amd as B
from oracle import constants as OC
from oracle import systems as S
from tests.bemutil import edge_perm, final_perm, rel

pytestmark = pytest.mark.gpu


def _row(eps):
    xyz, tri, obj = meshgen.sphere_row(1, 3, 0.5)
    khat, pol = meshgen.plane_wave_draws(1, 29)
    return meshgen.Workload("ico80x3", xyz, tri, obj, meshgen.freq_from_k0(1.5), list(eps), [1.0] * 3, [0.0] * 3,
                            eps_bg=1.2 - 0.02j, khat=khat, pol=pol.astype(np.complex128))


CASES = {
    "ico80x3_same": (lambda: _row([3.0 - 0.05j] * 3), 1),
    "ico80x3_mixed": (lambda: _row([3.0 - 0.05j, 6.0, 3.0 - 0.05j]), 2),
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


_oracle, _ops = {}, {}


def case(name, ctx, reuse=True, precision=B.BEM_FP64, formulation=B.BEM_FORM_SLDM, inner=B.BEM_INNER_AUTO):
    key = (name, reuse, precision, formulation, inner)
    if key in _ops:
        return _ops[key]
    w = CASES[name][0]()
    if name not in _oracle:
        _oracle[name] = S.assemble(w.xyz, w.tri, w.obj, S.Problem(w.freq_hz, w.eps_r, w.mu_r, w.sigma, eps_bg=w.eps_bg))
    ops = _oracle[name]
    mesh = B.bem_mesh_load(ctx, w.xyz, w.tri, w.obj)
    op = B.bem_assemble(ctx, mesh, B.make_problem(w.freq_hz, w.eps_r, w.mu_r, w.sigma, eps_bg=w.eps_bg,
                                                  precision=precision, formulation=formulation, reuse=reuse,
                                                  inner_mode=inner))
    va, vb, _, _ = B.bem_edge_table(ctx, mesh)
    _ops[key] = (w, ops, op, edge_perm(va, vb, ops.topo.edges))
    return _ops[key]


@pytest.mark.parametrize("name", list(CASES))
def test_shared_blocks_match_oracle(name, ctx):
    w, ops, op, perm = case(name, ctx)
    st = B.bem_op_stats_get(ctx, op)
    assert st["interiors_filled"] == CASES[name][1]
    _, _, op_all, _ = case(name, ctx, reuse=False)
    st_all = B.bem_op_stats_get(ctx, op_all)
    assert st_all["interiors_filled"] == 3
    print(f"{name}: device bytes shared {st['device_bytes'] / 1e6:.2f} MB, unshared {st_all['device_bytes'] / 1e6:.2f} MB")
    assert st["device_bytes"] < st_all["device_bytes"]
    ne, nt = len(ops.topo.edges), len(ops.topo.tri)
    blocks = {B.BEM_BLOCK_LA_INT: ops.LA_int, B.BEM_BLOCK_LPHI_INT: ops.Lphi_int, B.BEM_BLOCK_K_INT: ops.K_int,
              B.BEM_BLOCK_K_BG: ops.K_bg, B.BEM_BLOCK_LA_BG: ops.LA_bg}
    for block, M in blocks.items():
        n = nt if block == B.BEM_BLOCK_LPHI_INT else ne
        G = B.bem_block_export(ctx, op, block, n, n)
        ref = M if block == B.BEM_BLOCK_LPHI_INT else M[np.ix_(perm, perm)]
        err = rel(G, ref)
        print(f"  block {block}: rel {err:.2e}")
        assert err < 1e-12, (block, err)


@pytest.mark.parametrize("inner", [B.BEM_INNER_DIRECT, B.BEM_INNER_SCHUR])
@pytest.mark.parametrize("name", list(CASES))
def test_final_product_matches_oracle(name, inner, ctx, torch_mod):
    torch = torch_mod
    w, ops, op, perm = case(name, ctx, inner=inner)
    ne, nq = len(ops.topo.edges), ops.B.shape[1]
    M = S.final_matrix(ops)
    P = final_perm(perm, ne, nq)
    ref_M = M[np.ix_(P, P)]
    rng = np.random.default_rng(23)
    for nrhs in (1, 5):
        x = rng.standard_normal((nrhs, len(M))) + 1j * rng.standard_normal((nrhs, len(M)))
        xd = torch.tensor(x, dtype=torch.complex128, device="cuda")
        yd = torch.zeros_like(xd)
        B.bem_apply(ctx, op, B.BEM_BLOCK_FINAL, xd.data_ptr(), yd.data_ptr(), nrhs,
                    torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        err = rel(yd.cpu().numpy(), x @ ref_M.T)
        print(f"{name} inner {inner} nrhs {nrhs}: rel {err:.2e}")
        assert err < 1e-11


@pytest.mark.parametrize("formulation", [B.BEM_FORM_SLDM, B.BEM_FORM_EAEFIE])
@pytest.mark.parametrize("precision", [B.BEM_FP64, B.BEM_MIXED])
@pytest.mark.parametrize("name", list(CASES))
def test_solve_matches_oracle_and_unshared(name, precision, formulation, ctx):
    w, ops, op, perm = case(name, ctx, precision=precision, formulation=formulation)
    ne, nt = len(ops.topo.edges), len(ops.topo.tri)
    fp64 = precision == B.BEM_FP64
    tol, bound = (1e-12, 1e-10) if fp64 else (1e-9, 1e-6)
    b = S.rhs(ops, w.khat[0], w.pol[0])
    if formulation == B.BEM_FORM_SLDM:
        ref = S.solve_augmented(ops, b)
        a, e, q = ref.a, ref.e, ref.q
    else:
        a, e, q = S.solve_final_eaefie(ops, b)
    want = (a / (1j * ops.k0), e * OC.ETA0, (ops.B @ q) / OC.C0)
    opts = B.solve_opts(tol=tol, restart=100, maxit=3000, inner_tol=1e-14, max_refine=8)
    rc, H, E, rho, info = B.bem_solve(ctx, op, B.plane_waves(w.khat, w.pol), opts, ne, nt)
    print(f"{name} prec {precision} form {formulation}: outer {info.outer_iters} res {info.rel_residual:.2e}")
    assert rc == B.BEM_OK
    for lab, got, ref_v in (("H", H[:, 0], want[0][perm]), ("E", E[:, 0], want[1][perm]), ("rho", rho[:, 0], want[2])):
        err = rel(got, ref_v)
        print(f"  {lab}: rel {err:.2e}")
        assert err < bound, (lab, err)
    if fp64:
        _, _, op_all, _ = case(name, ctx, reuse=False, precision=precision, formulation=formulation)
        rc2, H2, E2, rho2, _ = B.bem_solve(ctx, op_all, B.plane_waves(w.khat, w.pol), opts, ne, nt)
        assert rc2 == B.BEM_OK
        for got, ref_v in ((H, H2), (E, E2), (rho, rho2)):
            assert rel(got, ref_v) < 1e-10
