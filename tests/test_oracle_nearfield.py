"""Pins of the oracle's near field (Sec. II-C, eqs. diffsources / diffsourcesdis; the probe-line
observable of Sec. IV-D): the Mie near-field series against Maxwell's equations and against the
already-pinned far-field amplitudes, the per-triangle moments against brute-force integration,
charge continuity of the differential sources, Maxwell's equations for the radiated field, the
far-zone limit against the far-field vector N, and the transparent object."""
from __future__ import annotations

import math

import numpy as np
import pytest

import meshgen
from oracle import constants as C
from oracle import mie
from oracle import nearfield as NF
from oracle import operators as O
from oracle import quadrature as Q
from oracle import systems as S

ETA0 = C.ETA0


def _jacobian(f, p, h):
    J = np.zeros((3, 3), complex)
    for j in range(3):
        e = np.zeros(3)
        e[j] = h
        J[:, j] = (f(p + e) - f(p - e)) / (2 * h)
    return J


def _curl(J):
    return np.array([J[2, 1] - J[1, 2], J[0, 2] - J[2, 0], J[1, 0] - J[0, 1]])


def test_mie_near_field_satisfies_maxwell():
    """curl E = -j k eta H, curl H = j (k / eta) E and zero divergences outside a lossy sphere
    (e^{+j omega t}); central differences, step 1e-4 a."""
    eps, a, k = 2.5 - 0.3j, 1.0, 1.7
    for p in (np.array([1.3, 0.2, 0.1]), np.array([-0.5, 0.9, -1.1]), np.array([0.1, 0.0, -2.0])):
        E, H = (v[0] for v in mie.near_field(eps, a, k, p))
        JE = _jacobian(lambda q: mie.near_field(eps, a, k, q)[0][0], p, 1e-4)
        JH = _jacobian(lambda q: mie.near_field(eps, a, k, q)[1][0], p, 1e-4)
        cE, cH = _curl(JE), _curl(JH)
        assert np.linalg.norm(cE + 1j * k * ETA0 * H) < 1e-6 * np.linalg.norm(cE)
        assert np.linalg.norm(cH - 1j * k / ETA0 * E) < 1e-6 * np.linalg.norm(cH)
        assert abs(np.trace(JE)) < 1e-6 * k * np.linalg.norm(E)
        assert abs(np.trace(JH)) < 1e-6 * k * np.linalg.norm(H)


def test_mie_near_field_far_zone():
    """At k r = 1e5 the series field is transverse, H = rhat x E / eta, and 4 pi r^2 |E|^2 is
    the bistatic RCS of the amplitude functions S1, S2 (an independent form of the series)."""
    eps, a, k, R = 4.0, 1.0, 1.0, 1e5
    for th in (0.3, 1.2, 2.5):
        for phi in (0.0, 0.7, math.pi / 2):
            rh = np.array([math.sin(th) * math.cos(phi), math.sin(th) * math.sin(phi), math.cos(th)])
            E, H = (v[0] for v in mie.near_field(eps, a, k, R * rh))
            s = 4 * math.pi * R * R * np.sum(np.abs(E) ** 2)
            assert abs(s / mie.bistatic_rcs(eps, a, k, th, phi)[0] - 1) < 1e-4
            assert abs(E @ rh) < 1e-3 * np.linalg.norm(E)
            assert np.linalg.norm(np.cross(rh, E) / ETA0 - H) < 1e-4 * np.linalg.norm(H)


TRI = np.array([[[0.0, 0.0, 0.0], [1.0, 0.1, 0.0], [0.3, 0.9, 0.05]]])


def _brute_moments(k, r):
    def f(rp):
        d = rp - r
        R = np.linalg.norm(d, axis=1)
        g, gg = O.green(k, R), O.grad_green_scalar(k, R)
        return np.concatenate([g[:, None], g[:, None] * d, gg[:, None] * (-d)], axis=1)
    return Q.brute_inner(f, r, TRI[0], order=24)


@pytest.mark.parametrize("k", [1.3, 2.0 - 0.4j])
def test_triangle_moments_against_brute_force(k):
    """I0, I1, Ig of one triangle at points 0.02-3 longest edges off its plane, inside and
    outside its outline, against graded Duffy Gauss-Legendre integration of the full kernels:
    the default rules within 1e-5 (singularity extraction for near points, the 7-point rule
    beyond twice the longest edge), and the extracted form with the remainder rule refined to
    level 4 within 1e-8 (so the closed-form static parts are exact)."""
    V = TRI
    h = O.longest_edge(V)[0]
    c = V[0].mean(0)
    n = np.cross(V[0, 1] - V[0, 0], V[0, 2] - V[0, 0])
    n /= np.linalg.norm(n)
    cases = [((0.1, 0.1), 0.02), ((0.0, 0.0), 0.3), ((0.5, -0.3), 0.1), ((1.2, 0.3), 0.05),
             ((0.0, 0.0), -0.2), ((0.0, 0.0), 1.5), ((0.2, 0.3), 2.2), ((0.0, 0.0), 3.0)]
    for (u, v), dist in cases:
        r = c + u * (V[0, 1] - V[0, 0]) + v * (V[0, 2] - V[0, 0]) + dist * h * n
        ref = _brute_moments(k, r)
        scale = np.max(np.abs(ref))
        got = np.concatenate([[x[0]] if x.ndim == 1 else x[0] for x in NF.triangle_moments(k, r, V)])
        err = np.max(np.abs(got - ref)) / scale
        assert err < 1e-5, (u, v, dist, err)
        if np.linalg.norm(r - c) < O.NEAR_FACTOR * h:
            fine = NF.triangle_moments(k, r, V, level=np.array([4]), near=np.array([True]))
            got = np.concatenate([[x[0]] if x.ndim == 1 else x[0] for x in fine])
            assert np.max(np.abs(got - ref)) / scale < 1e-8, (u, v, dist)


def _small_sphere(eps=4.0, k0a=1.0, eps_bg=1.0, level=1):
    w = meshgen.sphere_workload(level, k0a, eps)
    prob = S.Problem(w.freq_hz, w.eps_r, w.mu_r, w.sigma, eps_bg=eps_bg)
    ops = S.assemble(w.xyz, w.tri, w.obj, prob)
    sol = S.solve_augmented(ops, S.rhs(ops, w.khat[0], w.pol[0]))
    return w, ops, sol


@pytest.fixture(scope="module")
def sphere80():
    return _small_sphere()


def test_differential_charge_obeys_continuity(sphere80):
    """rho_Delta = B (q - q_eq)/c0 equals -div J_Delta / (j omega) triangle by triangle (the
    continuity rows of the internal and equivalent problems), to round-off."""
    _, ops, sol = sphere80
    jd, rd = NF.differential_sources(ops, sol)
    want = -(ops.D @ jd) / (1j * ops.k0 * C.C0)
    assert np.linalg.norm(rd - want) < 1e-12 * np.linalg.norm(rd)


def test_radiated_field_satisfies_maxwell(sphere80):
    """Outside twice the longest edge from every centroid (one fixed rule for all triangles,
    smooth in r): curl E = -j omega mu H and curl H = j omega eps E to the difference step's
    accuracy; div E = 0 up to the rule's error (it holds through charge continuity, so a wrong
    charge term would leave an O(1) divergence)."""
    w, ops, sol = sphere80
    jd, rd = NF.differential_sources(ops, sol)
    k = ops.k_bg
    for p in (np.array([2.3, 0.4, -0.2]), np.array([-0.3, -1.9, 1.4])):
        E, H = (v[0] for v in NF.radiated_field(ops, jd, rd, p))
        JE = _jacobian(lambda q: NF.radiated_field(ops, jd, rd, q)[0][0], p, 1e-4)
        JH = _jacobian(lambda q: NF.radiated_field(ops, jd, rd, q)[1][0], p, 1e-4)
        cE, cH = _curl(JE), _curl(JH)
        assert np.linalg.norm(cE + 1j * k * ETA0 * H) < 1e-6 * np.linalg.norm(cE)
        assert np.linalg.norm(cH - 1j * k / ETA0 * E) < 1e-3 * np.linalg.norm(cH)
        assert abs(np.trace(JE)) < 1e-3 * abs(k) * np.linalg.norm(E)


def test_far_zone_limit_is_the_far_field(sphere80):
    """E(R rhat) R e^{j k R} -> -j omega mu / (4 pi) N_perp(rhat) and H -> rhat x E / eta as
    R grows, N from the far-field routine (its own phase-factor form of the same current)."""
    _, ops, sol = sphere80
    jd, rd = NF.differential_sources(ops, sol)
    R = 1e6
    rh = np.array([[0.0, 0.0, 1.0], [0.6, 0.0, -0.8], [0.0, 1.0, 0.0], [0.48, 0.6, 0.64]])
    N = S.far_field_N(ops, jd, rh)
    E, H = NF.radiated_field(ops, jd, rd, R * rh)
    jwmu = 1j * ops.k0 * C.C0 * C.MU0
    for d in range(len(rh)):
        Np = N[d] - (N[d] @ rh[d]) * rh[d]
        want = -jwmu / (4 * math.pi) * Np
        got = E[d] * R * np.exp(1j * ops.k_bg * R)
        assert np.linalg.norm(got - want) < 1e-5 * np.linalg.norm(want), d
        assert np.linalg.norm(np.cross(rh[d], E[d]) / ETA0 - H[d]) < 1e-5 * np.linalg.norm(H[d])


def test_transparent_object_radiates_nothing():
    """eps_c = eps_l: J_Delta and rho_Delta vanish, so does the scattered near field."""
    w = meshgen.sphere_workload(1, 1.5, 2.0)
    prob = S.Problem(w.freq_hz, [2.0 - 0.3j], [1.0], [0.0], eps_bg=2.0 - 0.3j)
    ops = S.assemble(w.xyz, w.tri, w.obj, prob)
    sol = S.solve_augmented(ops, S.rhs(ops, w.khat[0], w.pol[0]))
    pts = np.array([[1.5, 0.0, 0.0], [0.0, -2.0, 0.5]])
    E, H = NF.near_field(ops, sol, pts)
    Ei, Hi = NF.incident_plane_wave(ops, w.khat[0], w.pol[0], pts)
    assert np.abs(E).max() < 1e-10 * np.abs(Ei).max()
    assert np.abs(H).max() < 1e-10 * np.abs(Hi).max()
