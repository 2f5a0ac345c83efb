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
from oracle import constants as OC
from oracle import systems as S
from tests.bemutil import edge_perm, final_perm, meq_perm, rel

pytestmark = pytest.mark.gpu

def _sphere(level, k0a, eps, eps_bg):
    def make():
        w = meshgen.sphere_workload(level, k0a, eps)
        w.eps_bg = eps_bg
        return w
    return make


def _ellipsoid_jittered():
    """Small counterpart of the batched-excitation ellipsoid: cubed sphere n = 5 (300
    triangles) on semi-axes 1/0.6/0.4 m with 2% seeded vertex jitter, eps_r = 6, k0 a = 2."""
    xyz, tri = meshgen.cubed_sphere(5, (1.0, 0.6, 0.4))
    xyz = meshgen.jitter(xyz, tri, 0.02, seed=3)
    khat, pol = meshgen.plane_wave_draws(1, 7)
    return meshgen.Workload("ell300_eps6_jitter", xyz, tri, np.zeros(len(tri), np.int32), meshgen.freq_from_k0(2.0),
                            [6.0], [1.0], [0.0], khat=khat, pol=pol.astype(np.complex128))


def _copper_bars():
    """Small counterpart of the conductor array: two copper bars (10 x 1 x 1 um, sigma =
    5.8e7 S/m, 176 triangles each, graded) 3 um apart in eps_r = 4, at 10 GHz; two objects,
    a skin depth below the bar thickness and |k_l| h ~ 1e-3 (augmented direct nested solve)."""
    bars = []
    for dy in (0.0, 3e-6):
        x, t, _ = meshgen.copper_bars(h_min=0.5e-6, h_max=2e-6, grid=1)
        x = x + np.array([0.0, dy, 0.0])
        bars.append((x, t))
    xyz, tri, obj = meshgen.merge(bars)
    w = meshgen.Workload("bars2_cu_10GHz", xyz, tri, obj, 1e10, [1.0, 1.0], [1.0, 1.0], [5.8e7, 5.8e7])
    w.eps_bg = 4.0
    return w


CASES = {
    "ico80_eps4": _sphere(1, 1.0, 4.0, 1.0),
    "ico80_lossy": _sphere(1, 2.0, 2.5 - 0.1j, 1.5 - 0.05j),
    "ell300_eps6_jitter": _ellipsoid_jittered,
    "bars2_cu_10GHz": _copper_bars,
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
    w = CASES[name]()
    if name not in _oracle:
        prob = S.Problem(w.freq_hz, w.eps_r, w.mu_r, w.sigma, eps_bg=w.eps_bg)
        _oracle[name] = S.assemble(w.xyz, w.tri, w.obj, prob)
    ops = _oracle[name]
    mesh = B.bem_mesh_load(ctx, w.xyz, w.tri, w.obj)
    p = B.make_problem(w.freq_hz, w.eps_r, w.mu_r, w.sigma, eps_bg=w.eps_bg, precision=precision, inner_mode=inner,
                       precond=precond)
    op = B.bem_assemble(ctx, mesh, p)
    va, vb, _, _ = B.bem_edge_table(ctx, mesh)
    perm = edge_perm(va, vb, ops.topo.edges)
    _cache[key] = (w, ops, mesh, op, perm)
    return _cache[key]


def test_device_inverse_of_meq(ctx):
    """The direct nested solve's device inverse times the oracle's M_eq is the identity (blocked
    Gauss-Jordan, panels applied in groups of four by the float64 4x4x4 matrix-core update).
    M_eq has 199 rows: one group of four panels, the last with 7 rows.  The assembly's own
    inversion health is reported in the operator statistics."""
    w = CASES["ico80_lossy"]()
    if "ico80_lossy" not in _oracle:
        _oracle["ico80_lossy"] = S.assemble(w.xyz, w.tri, w.obj,
                                            S.Problem(w.freq_hz, w.eps_r, w.mu_r, w.sigma, eps_bg=w.eps_bg))
    ops = _oracle["ico80_lossy"]
    mesh = B.bem_mesh_load(ctx, w.xyz, w.tri)
    op = B.bem_assemble(ctx, mesh, B.make_problem(w.freq_hz, w.eps_r, w.mu_r, w.sigma, eps_bg=w.eps_bg,
                                                  inner_mode=B.BEM_INNER_DIRECT, precond=0))
    va, vb, _, _ = B.bem_edge_table(ctx, mesh)
    perm = edge_perm(va, vb, ops.topo.edges)
    ne, nt = len(ops.topo.edges), len(ops.topo.tri)
    Meq, _, _ = S.equivalent_matrix_object(ops, 0)
    P = meq_perm(perm, ne, nt - 1)
    Minv = B.bem_block_export(ctx, op, B.BEM_BLOCK_MEQ_INV, len(Meq), len(Meq))
    err = np.abs(Minv @ Meq[np.ix_(P, P)] - np.eye(len(Meq))).max()
    st = B.bem_op_stats_get(ctx, op)
    print(f"max |M_eq^-1 M_eq - I| = {err:.2e}; pivot ratio {st['inverse_min_pivot_ratio']:.2e}, "
          f"probe error {st['inverse_probe_error']:.2e}")
    B.bem_release(ctx, op)
    assert err < 1e-10
    assert st["inverse_min_pivot_ratio"] > 1e-6 and st["inverse_probe_error"] < 1e-12


def full_meq(ops):
    """Block-diagonal M_eq of all objects, ordered [all edges; all kept charges]."""
    ne, nq = len(ops.topo.edges), ops.B.shape[1]
    M = np.zeros((ne + nq, ne + nq), complex)
    for o in range(ops.topo.n_obj):
        Mo, e_idx, q_idx = S.equivalent_matrix_object(ops, o)
        idx = np.concatenate([e_idx, ne + q_idx])
        M[np.ix_(idx, idx)] = Mo
    return M


def schur_ok(name):
    """Charge elimination is used while |k_l| h >= 0.01 (the conductor case is below)."""
    return name != "bars2_cu_10GHz"


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
    nq = ops.B.shape[1]
    rng = np.random.default_rng(7)
    B.bem_set_inner_tol(ctx, op, 1e-14)
    blocks = oracle_blocks(ops)
    blocks[B.BEM_BLOCK_MEQ] = full_meq(ops)
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
    if inner == B.BEM_INNER_SCHUR and not schur_ok(name):
        pytest.skip("charge elimination is not used at |k h| < 0.01")
    torch = torch_mod
    w, ops, mesh, op, perm = case(name, ctx, inner, 0)
    ne, nt = len(ops.topo.edges), len(ops.topo.tri)
    M = S.final_matrix(ops)
    P = final_perm(perm, ne, ops.B.shape[1])
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


SMALL = ("ico80_eps4", "ico80_lossy")

# (float64 solve tolerance, float64 parity bound, mixed solve tolerance, mixed parity bound).
# The conductor case at |k_l h| ~ 1e-3 is a conditioning limit, measured on the oracle's
# matrices for the port excitation: the terms of the final system cancel (|| |A| |x| || / ||b||
# = 1.1e7), so float64 products carry ~2e-9 relative residual noise and LAPACK's own solution
# has residual 4.6e-10; two float64 LU solves of the augmented system that differ only in the
# elimination order disagree by 1e-8 (H) to 3e-8 (E).  1e-7 is the smallest residual certified
# reliably there, and 1e-6 the currents' bound at that residual.
TOLS = {"bars2_cu_10GHz": (1e-7, 1e-6, 1e-7, 1e-6)}
DEFAULT_TOLS = (1e-12, 1e-10, 1e-9, 1e-6)
# The conductor array is driven by ports; a plane wave on a 10 um structure at 10 GHz induces
# currents 1e-9 of the port case, set by cancellations the float64 residual cannot resolve.
PORT_ONLY = ("bars2_cu_10GHz",)


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("inner,precond", MODES)
def test_solve_fp64_matches_oracle(name, inner, precond, ctx):
    if inner == B.BEM_INNER_SCHUR and not schur_ok(name):
        pytest.skip("charge elimination is not used at |k h| < 0.01")
    if precond == 0 and name not in SMALL:
        pytest.skip("unpreconditioned runs are checked on the 80-triangle cases only")
    if name in PORT_ONLY:
        pytest.skip("port-driven case: see test_delta_gap_port_on_conductors")
    w, ops, mesh, op, perm = case(name, ctx, inner, precond)
    ne, nt = len(ops.topo.edges), len(ops.topo.tri)
    stol, bound, _, _ = TOLS.get(name, DEFAULT_TOLS)
    b = S.rhs(ops, w.khat[0], w.pol[0])
    ref = S.solve_augmented(ops, b)
    exc = B.plane_waves(w.khat, w.pol)
    rc, H, E, rho, info = B.bem_solve(ctx, op, exc, B.solve_opts(tol=stol, restart=100, maxit=3000,
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
        assert err < bound, (lab, err)


@pytest.mark.parametrize("inner", [B.BEM_INNER_DIRECT, B.BEM_INNER_SCHUR])
@pytest.mark.parametrize("name", list(CASES))
def test_solve_mixed_matches_oracle(name, inner, ctx):
    """float32 products and nested solves, float64 Arnoldi and residual refinement: after
    refinement to a 1e-9 float64 residual the currents are within 1e-6 of the oracle."""
    if inner == B.BEM_INNER_SCHUR and not schur_ok(name):
        pytest.skip("charge elimination is not used at |k h| < 0.01")
    if name in PORT_ONLY:
        pytest.skip("port-driven case: see test_delta_gap_port_on_conductors")
    w, ops, mesh, op, perm = case(name, ctx, inner, 1, B.BEM_MIXED)
    ne, nt = len(ops.topo.edges), len(ops.topo.tri)
    _, _, mtol, bound = TOLS.get(name, DEFAULT_TOLS)
    ref = S.solve_augmented(ops, S.rhs(ops, w.khat[0], w.pol[0]))
    rc, H, E, rho, info = B.bem_solve(ctx, op, B.plane_waves(w.khat, w.pol),
                                      B.solve_opts(tol=mtol, restart=100, maxit=3000, max_refine=8), ne, nt)
    print(f"{name} mixed: outer {info.outer_iters} refine {info.refine_steps} res {info.rel_residual:.2e}")
    assert rc == B.BEM_OK and info.rel_residual <= mtol
    for lab, got, want in (("H", H[:, 0], ref.H(ops.k0)[perm]), ("E", E[:, 0], ref.E()[perm]),
                           ("rho", rho[:, 0], ref.rho(ops.B))):
        err = rel(got, want)
        print(f"  {lab}: rel {err:.2e}")
        assert err < bound, (lab, err)


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
    if name in PORT_ONLY:
        pytest.skip("port-driven case: see test_delta_gap_port_on_conductors")
    w, ops, mesh, op, perm = case(name, ctx, B.BEM_INNER_SCHUR, 1, precision)
    ne, nt = len(ops.topo.edges), len(ops.topo.tri)
    khat, pol, refs = _multi_reference(ops, N_EXC, 5)
    fp64 = precision == B.BEM_FP64
    stol, sbound, mtol, mbound = TOLS.get(name, DEFAULT_TOLS)
    opts = B.solve_opts(tol=stol if fp64 else mtol, restart=60, maxit=3000, max_refine=8)
    rc, H, E, rho, info = B.bem_solve(ctx, op, B.plane_waves(khat, pol), opts, ne, nt)
    print(f"{name} prec {precision}: outer {info.outer_iters} refine {info.refine_steps} "
          f"products {info.n_products} res {info.rel_residual:.2e}")
    assert rc == B.BEM_OK
    tol = sbound if fp64 else mbound
    for c, ref in enumerate(refs):
        for lab, got, want in (("H", H[:, c], ref.H(ops.k0)[perm]), ("E", E[:, c], ref.E()[perm]),
                               ("rho", rho[:, c], ref.rho(ops.B))):
            err = rel(got, want)
            assert err < tol, (c, lab, err)


@pytest.mark.parametrize("precision", [B.BEM_FP64, B.BEM_MIXED])
def test_delta_gap_port_on_conductors(precision, ctx):
    """Port-like voltage gap on the first copper bar: the edges of the ring x = 0 are driven
    with b_m = +V/eta0 for the pair (a, b) = (va, vb) of edge m (the right-hand side is built
    here from that definition).  Currents of both bars match the oracle's direct solve to the
    bounds of TOLS (float32 sweeps that stall hand over to float64 products)."""
    w, ops, mesh, op, perm = case("bars2_cu_10GHz", ctx, B.BEM_INNER_AUTO, 1, precision)
    topo = ops.topo
    ne, nt = len(topo.edges), len(topo.tri)
    x = topo.xyz[:, 0]
    ring = [i for i, (a, b) in enumerate(topo.edges)
            if topo.edge_obj[i] == 0 and abs(x[a]) < 1e-12 and abs(x[b]) < 1e-12]
    assert len(ring) >= 8
    pairs = np.array([topo.edges[i] for i in ring], np.int32)
    b = np.zeros(ne, complex)
    b[ring] = 1.0 / OC.ETA0
    ref = S.solve_augmented(ops, b)
    fp64 = precision == B.BEM_FP64
    stol, sbound, mtol, mbound = TOLS["bars2_cu_10GHz"]
    rc, H, E, rho, info = B.bem_solve(ctx, op, B.delta_gaps([pairs]),
                                      B.solve_opts(tol=stol if fp64 else mtol, restart=200, maxit=4000,
                                                   inner_tol=1e-14 if fp64 else 0.0, max_refine=8), ne, nt)
    print(f"delta gap prec {precision}: outer {info.outer_iters} refine {info.refine_steps} "
          f"res {info.rel_residual:.2e}")
    assert rc == B.BEM_OK
    tol = sbound if fp64 else mbound
    for lab, got, want in (("H", H[:, 0], ref.H(ops.k0)[perm]), ("E", E[:, 0], ref.E()[perm]),
                           ("rho", rho[:, 0], ref.rho(ops.B))):
        err = rel(got, want)
        print(f"  {lab}: rel {err:.2e}")
        assert err < tol, (lab, err)
