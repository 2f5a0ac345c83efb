"""Near field of device solutions (bem_near_field): E and H at exterior points radiated by the
differential current and charge in the background (Sec. II-C; the probe-line observable of
Sec. IV-D).  Against the oracle's near field element by element on small cases (one sphere; two
spheres in a lossy background; 5 plane waves, so the 4-column groups are ragged; points from
just off the surface, where the singularity-extracted form runs, out to three radii), the total
field against scattered plus incident, the far-zone limit against bem_far_field, at full size
(5120 triangles) against the Mie series, and the argument checks."""
from __future__ import annotations

import math

import numpy as np
import pytest

import meshgen
import paper_2106_06184_amd as B
from oracle import constants as C
from oracle import mie
from oracle import nearfield as NF
from oracle import systems as S
from tests.bemutil import edge_perm, rel

pytestmark = pytest.mark.gpu


def _points(n, rmin, rmax, seed, centre=(0.0, 0.0, 0.0)):
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return np.asarray(centre) + d * np.linspace(rmin, rmax, n)[:, None]


def _two_lossy():
    xyz, tri, obj = meshgen.sphere_row(1, 2, 0.4)
    khat, pol = meshgen.plane_wave_draws(5, 43)
    return meshgen.Workload("two_ico80", xyz, tri, obj, meshgen.freq_from_k0(1.2), [4.0, 2.5 - 0.3j], [1.0, 1.0],
                            [0.0, 0.0], eps_bg=1.3 - 0.01j, khat=khat, pol=pol.astype(np.complex128))


def _one():
    w = meshgen.sphere_workload(1, 1.0, 4.0)
    khat, pol = meshgen.plane_wave_draws(5, 44)
    return meshgen.Workload("ico80", w.xyz, w.tri, w.obj, w.freq_hz, w.eps_r, w.mu_r, w.sigma, eps_bg=w.eps_bg,
                            khat=khat, pol=pol.astype(np.complex128))


def _exterior(w, n, seed):
    """Points outside every sphere of the workload, some within a triangle size of a surface."""
    obj = np.asarray(w.obj)
    centres = np.array([w.xyz[np.unique(w.tri[obj == o])].mean(axis=0) for o in range(obj.max() + 1)])
    radius = max(np.linalg.norm(w.xyz[np.unique(w.tri[obj == o])] - centres[o], axis=1).max()
                 for o in range(len(centres)))
    pts = []
    rng = np.random.default_rng(seed)
    while len(pts) < n:
        o = rng.integers(len(centres))
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        p = centres[o] + d * radius * rng.uniform(1.08, 3.0)
        if np.all(np.linalg.norm(centres - p, axis=1) > 1.05 * radius):
            pts.append(p)
    return np.array(pts)


CASES = {"ico80_eps4": _one, "two_ico80_lossy_bg": _two_lossy}


@pytest.fixture(scope="module")
def ctx():
    c = B.bem_create(0)
    yield c
    B.bem_destroy(c)


@pytest.mark.parametrize("name", list(CASES))
def test_near_field_matches_oracle(name, ctx):
    """Oracle solution (augmented LU) fed to the device: its equivalent solve and near-field
    kernel against the oracle's near field of the same solution, within 1e-12; the device's own
    solve (tol 1e-12) end to end within 1e-10."""
    w = CASES[name]()
    ops = S.assemble(w.xyz, w.tri, w.obj, S.Problem(w.freq_hz, w.eps_r, w.mu_r, w.sigma, eps_bg=w.eps_bg))
    mesh = B.bem_mesh_load(ctx, w.xyz, w.tri, w.obj)
    info = B.bem_mesh_info(ctx, mesh)
    op = B.bem_assemble(ctx, mesh, B.make_problem(w.freq_hz, w.eps_r, w.mu_r, w.sigma, eps_bg=w.eps_bg))
    B.bem_set_inner_tol(ctx, op, 1e-14)
    va, vb, _, _ = B.bem_edge_table(ctx, mesh)
    perm = edge_perm(va, vb, ops.topo.edges)
    pts = _exterior(w, 37, 7)
    R = len(w.khat)
    sols = [S.solve_augmented(ops, S.rhs(ops, w.khat[c], w.pol[c])) for c in range(R)]
    Hq = np.stack([s.H(ops.k0)[perm] for s in sols], 1)
    Eq = np.stack([s.E()[perm] for s in sols], 1)
    rq = np.stack([s.rho(ops.B) for s in sols], 1)
    Eg, Hg = B.bem_near_field(ctx, op, Hq, Eq, rq, pts)
    rc, H, E, rho, _ = B.bem_solve(ctx, op, B.plane_waves(w.khat, w.pol),
                                   B.solve_opts(tol=1e-12, restart=100, maxit=3000, inner_tol=1e-14),
                                   info["n_edge"], info["n_tri"])
    assert rc == B.BEM_OK
    Ed, Hd = B.bem_near_field(ctx, op, H, E, rho, pts)
    for c in range(R):
        Er, Hr = NF.near_field(ops, sols[c], pts)
        e1, e2 = max(rel(Eg[c], Er), rel(Hg[c], Hr)), max(rel(Ed[c], Er), rel(Hd[c], Hr))
        print(f"{name} exc {c}: oracle solution {e1:.2e}, device solution {e2:.2e}")
        assert e1 < 1e-12 and e2 < 1e-10
    # bitwise reproducible
    Eg2, Hg2 = B.bem_near_field(ctx, op, Hq, Eq, rq, pts)
    assert np.array_equal(Eg, Eg2) and np.array_equal(Hg, Hg2)
    B.bem_release(ctx, op)


def test_total_field_and_far_zone(ctx):
    """With the plane waves given, the output is the scattered field plus E0 pol e^{-jk khat.r}
    and khat x E / eta; at R = 1e6 the scattered field is -j omega mu e^{-jkR}/(4 pi R) N_perp
    of bem_far_field."""
    w = _two_lossy()
    mesh = B.bem_mesh_load(ctx, w.xyz, w.tri, w.obj)
    info = B.bem_mesh_info(ctx, mesh)
    op = B.bem_assemble(ctx, mesh, B.make_problem(w.freq_hz, w.eps_r, w.mu_r, w.sigma, eps_bg=w.eps_bg))
    exc = B.plane_waves(w.khat, w.pol)
    rc, H, E, rho, _ = B.bem_solve(ctx, op, exc, B.solve_opts(tol=1e-10, restart=100, maxit=3000),
                                   info["n_edge"], info["n_tri"])
    assert rc == B.BEM_OK
    pts = _exterior(w, 11, 8)
    Es, Hs = B.bem_near_field(ctx, op, H, E, rho, pts)
    Et, Ht = B.bem_near_field(ctx, op, H, E, rho, pts, exc=exc)
    k = 2 * math.pi * w.freq_hz / C.C0 * np.sqrt(complex(w.eps_bg))
    if k.imag > 0:
        k = -k
    eta = C.ETA0 / np.sqrt(complex(w.eps_bg))
    for c in range(len(w.khat)):
        Ei = w.pol[c][None, :] * np.exp(-1j * k * (pts @ w.khat[c]))[:, None]
        Hi = np.cross(np.broadcast_to(w.khat[c], Ei.shape), Ei) / eta
        assert rel(Et[c] - Es[c], Ei) < 1e-12 and rel(Ht[c] - Hs[c], Hi) < 1e-12
    rh = np.array([[0.0, 0.0, 1.0], [0.6, 0.0, -0.8], [0.48, 0.6, 0.64]])
    Rf = 1e6
    N, _ = B.bem_far_field(ctx, op, H, E, rh)
    Ef, Hf = B.bem_near_field(ctx, op, H, E, rho, Rf * rh)
    jwmu = 1j * 2 * math.pi * w.freq_hz * C.MU0
    for c in range(len(w.khat)):
        for d in range(len(rh)):
            Np = N[c, d] - (N[c, d] @ rh[d]) * rh[d]
            want = -jwmu / (4 * math.pi) * Np * np.exp(-1j * k * Rf) / Rf
            assert rel(Ef[c, d], want) < 1e-5, (c, d)
    B.bem_release(ctx, op)


def test_full_size_near_field_against_mie(ctx):
    """The 5120-triangle sphere (eps_r = 4, k0 a = 1), 200 points between 1.2 and 3 radii in
    groups of 4 columns (one plane wave), against the Mie series: the discretisation error, 3.5%
    at 320 triangles in the oracle, falls below 0.6% here."""
    w = meshgen.sphere_workload(4, 1.0, 4.0)
    mesh = B.bem_mesh_load(ctx, w.xyz, w.tri)
    info = B.bem_mesh_info(ctx, mesh)
    op = B.bem_assemble(ctx, mesh, B.make_problem(w.freq_hz, w.eps_r, w.mu_r, w.sigma))
    rc, H, E, rho, _ = B.bem_solve(ctx, op, B.plane_waves(w.khat[:1], w.pol[:1]),
                                   B.solve_opts(tol=1e-10, restart=200, maxit=3000), info["n_edge"], info["n_tri"])
    assert rc == B.BEM_OK
    pts = _points(200, 1.2, 3.0, 9)
    Ed, Hd = B.bem_near_field(ctx, op, H, E, rho, pts)
    Em, Hm = mie.near_field(4.0, 1.0, 2 * math.pi * w.freq_hz / C.C0, pts)
    eE, eH = rel(Ed[0], Em), rel(Hd[0], Hm)
    print(f"5120 triangles vs Mie: E {eE:.2e}, H {eH:.2e}")
    assert eE < 6e-3 and eH < 6e-3
    B.bem_release(ctx, op)


def test_argument_checks(ctx):
    w = _one()
    mesh = B.bem_mesh_load(ctx, w.xyz, w.tri)
    info = B.bem_mesh_info(ctx, mesh)
    op = B.bem_assemble(ctx, mesh, B.make_problem(w.freq_hz, w.eps_r, w.mu_r, w.sigma))
    rc, H, E, rho, _ = B.bem_solve(ctx, op, B.plane_waves(w.khat[:1], w.pol[:1]), B.solve_opts(tol=1e-8),
                                   info["n_edge"], info["n_tri"])
    Ez, Hz = B.bem_near_field(ctx, op, H, E, rho, np.zeros((0, 3)))
    assert Ez.shape == (1, 0, 3) and Hz.shape == (1, 0, 3)
    with pytest.raises(B.BemError) as ei:
        B.bem_near_field(ctx, op, H, E, rho, np.array([[np.nan, 0.0, 2.0]]))
    assert "status -1" in str(ei.value)
    gap = B.delta_gaps([np.array([[int(w.tri[0, 0]), int(w.tri[0, 1])]])])
    with pytest.raises(B.BemError) as ei:
        B.bem_near_field(ctx, op, H, E, rho, np.array([[0.0, 0.0, 2.0]]), exc=gap)
    assert "status -1" in str(ei.value)
    ea = B.bem_assemble(ctx, mesh, B.make_problem(w.freq_hz, w.eps_r, w.mu_r, w.sigma,
                                                  formulation=B.BEM_FORM_EAEFIE))
    with pytest.raises(B.BemError) as ei:
        B.bem_near_field(ctx, ea, H, E, rho, np.array([[0.0, 0.0, 2.0]]))
    assert "status -1" in str(ei.value)
