"""GPU parity where the source rules are subdivided (highly conductive objects): an 80-triangle
sphere of sigma = 0.5 S/m at k0 = 1 (|Re k| h = 6 for its triangles: level 2 for L, level 1-2
for the barycentric pieces of K~), and a 320-triangle sphere at a skin depth of a quarter of
its edges.  Blocks at 1e-12 (K~ at 1e-11: at |k| R >= 0.5 its near remainder
g_k + 1/(4 pi R^3) + k^2/(8 pi R) is formed from terms up to (|k| R)^-3 ~ 8 times larger than
the result, so the two sides' rounding differs by more there), the final product at 1e-11 and
the float64 solve at 1e-10 against the oracle (which subdivides by the same rule)."""
from __future__ import annotations

import numpy as np
import pytest

import meshgen
import paper_2106_06184_amd as B
from oracle import operators as OO
from oracle import systems as S
from tests.bemutil import edge_perm, final_perm, rel

pytestmark = pytest.mark.gpu


def _conductor_sphere(level, sigma):
    w = meshgen.sphere_workload(level, 1.0, 1.0)
    w.sigma = [sigma]
    return w


CASES = {"ico80_sigma0.5": lambda: _conductor_sphere(1, 0.5), "ico320_sigma2": lambda: _conductor_sphere(2, 2.0)}


@pytest.fixture(scope="module")
def ctx():
    c = B.bem_create(0)
    yield c
    B.bem_destroy(c)


_ops = {}


def case(name, ctx):
    if name in _ops:
        return _ops[name]
    w = CASES[name]()
    ops = S.assemble(w.xyz, w.tri, w.obj, S.Problem(w.freq_hz, w.eps_r, w.mu_r, w.sigma))
    lev = OO.subdivision_level(ops.k_int[0], OO.longest_edge(OO.tri_vertices(ops.topo)))
    assert lev.min() >= 1, "the case must exercise the subdivided rules"
    mesh = B.bem_mesh_load(ctx, w.xyz, w.tri, w.obj)
    op = B.bem_assemble(ctx, mesh, B.make_problem(w.freq_hz, w.eps_r, w.mu_r, w.sigma, inner_mode=B.BEM_INNER_DIRECT))
    va, vb, _, _ = B.bem_edge_table(ctx, mesh)
    _ops[name] = (w, ops, op, edge_perm(va, vb, ops.topo.edges))
    return _ops[name]


@pytest.mark.parametrize("name", list(CASES))
def test_interior_blocks_match_oracle(name, ctx):
    w, ops, op, perm = case(name, ctx)
    ne, nt = len(ops.topo.edges), len(ops.topo.tri)
    for block, M in ((B.BEM_BLOCK_LA_INT, ops.LA_int), (B.BEM_BLOCK_LPHI_INT, ops.Lphi_int),
                     (B.BEM_BLOCK_K_INT, ops.K_int)):
        n = nt if block == B.BEM_BLOCK_LPHI_INT else ne
        G = B.bem_block_export(ctx, op, block, n, n)
        ref = M if block == B.BEM_BLOCK_LPHI_INT else M[np.ix_(perm, perm)]
        err = rel(G, ref)
        print(f"{name} block {block}: rel {err:.2e}")
        assert err < (1e-11 if block == B.BEM_BLOCK_K_INT else 1e-12), (block, err)


@pytest.mark.parametrize("name", list(CASES))
def test_final_product_and_solve_match_oracle(name, ctx):
    import torch
    w, ops, op, perm = case(name, ctx)
    ne, nt, nq = len(ops.topo.edges), len(ops.topo.tri), ops.B.shape[1]
    M = S.final_matrix(ops)
    P = final_perm(perm, ne, nq)
    rng = np.random.default_rng(31)
    x = rng.standard_normal((2, len(M))) + 1j * rng.standard_normal((2, len(M)))
    xd = torch.tensor(x, dtype=torch.complex128, device="cuda")
    yd = torch.zeros_like(xd)
    B.bem_apply(ctx, op, B.BEM_BLOCK_FINAL, xd.data_ptr(), yd.data_ptr(), 2, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    err = rel(yd.cpu().numpy(), x @ M[np.ix_(P, P)].T)
    print(f"{name} final product: rel {err:.2e}")
    assert err < 1e-11
    ref = S.solve_augmented(ops, S.rhs(ops, w.khat[0], w.pol[0]))
    rc, H, E, rho, info = B.bem_solve(ctx, op, B.plane_waves(w.khat, w.pol),
                                      B.solve_opts(tol=1e-12, restart=100, maxit=3000), ne, nt)
    print(f"{name} solve: outer {info.outer_iters} res {info.rel_residual:.2e}")
    assert rc == B.BEM_OK
    for lab, got, want in (("H", H[:, 0], ref.H(ops.k0)[perm]), ("E", E[:, 0], ref.E()[perm]),
                           ("rho", rho[:, 0], ref.rho(ops.B))):
        e = rel(got, want)
        print(f"  {lab}: rel {e:.2e}")
        assert e < 1e-10, (lab, e)
