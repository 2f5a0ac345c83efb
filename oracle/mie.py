"""Mie series for a homogeneous dielectric sphere (oracle; test infrastructure only).

The paper validates its sphere example against the Mie series (Sec. IV-A).
Textbook form (Bohren & Huffman, ch. 4) in the e^{-i omega t} convention: the
e^{+j omega t} permittivity eps_r - j eps'' of this code base is conj() first.
Only magnitudes (cross sections) are compared, which do not depend on the
time convention.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import special


def coefficients(m: complex, x: float, nmax: int | None = None):
    """a_n, b_n (n = 1..nmax) for relative index m and size parameter x (mu = 1)."""
    if nmax is None:
        nmax = int(round(x + 4 * x ** (1 / 3) + 2)) + 4
    n = np.arange(1, nmax + 1)
    mx = m * x
    jx = special.spherical_jn(n, x)
    djx = special.spherical_jn(n, x, derivative=True)
    yx = special.spherical_yn(n, x)
    dyx = special.spherical_yn(n, x, derivative=True)
    jmx = special.spherical_jn(n, mx)
    djmx = special.spherical_jn(n, mx, derivative=True)
    psi_x, dpsi_x = x * jx, jx + x * djx
    xi_x, dxi_x = x * (jx + 1j * yx), (jx + 1j * yx) + x * (djx + 1j * dyx)
    psi_mx, dpsi_mx = mx * jmx, jmx + mx * djmx
    a = (m * psi_mx * dpsi_x - psi_x * dpsi_mx) / (m * psi_mx * dxi_x - xi_x * dpsi_mx)
    b = (psi_mx * dpsi_x - m * psi_x * dpsi_mx) / (psi_mx * dxi_x - m * xi_x * dpsi_mx)
    return a, b


def angular(nmax: int, theta: np.ndarray):
    """pi_n, tau_n for n = 1..nmax at scattering angles theta (rows = n)."""
    mu = np.cos(theta)
    pi = np.zeros((nmax + 1, len(theta)))
    tau = np.zeros((nmax + 1, len(theta)))
    pi[1] = 1.0
    tau[1] = mu
    for n in range(2, nmax + 1):
        pi[n] = (2 * n - 1) / (n - 1) * mu * pi[n - 1] - n / (n - 1) * pi[n - 2]
        tau[n] = n * mu * pi[n] - (n + 1) * pi[n - 1]
    return pi[1:], tau[1:]


def amplitudes(m: complex, x: float, theta: np.ndarray):
    """S1, S2 at scattering angle theta (0 = forward)."""
    a, b = coefficients(m, x)
    nmax = len(a)
    n = np.arange(1, nmax + 1)
    pi, tau = angular(nmax, np.atleast_1d(theta))
    f = ((2 * n + 1) / (n * (n + 1)))[:, None]
    S1 = np.sum(f * (a[:, None] * pi + b[:, None] * tau), axis=0)
    S2 = np.sum(f * (a[:, None] * tau + b[:, None] * pi), axis=0)
    return S1, S2


def efficiencies(m: complex, x: float):
    a, b = coefficients(m, x)
    n = np.arange(1, len(a) + 1)
    qext = 2 / x ** 2 * np.sum((2 * n + 1) * (a + b).real)
    qsca = 2 / x ** 2 * np.sum((2 * n + 1) * (np.abs(a) ** 2 + np.abs(b) ** 2))
    qback = np.abs(np.sum((2 * n + 1) * (-1.0) ** n * (a - b))) ** 2 / x ** 2
    return qext, qsca, qback


def bistatic_rcs(eps_r: complex, radius: float, k_bg: float, theta_obs, phi_obs):
    """sigma(theta, phi) for a plane wave travelling along -z polarised along x,
    observed in direction (theta, phi) of the usual spherical angles.

    The scattering angle is pi - theta.  sigma = 4 pi / k^2 (|S2|^2 cos^2 phi + |S1|^2 sin^2 phi)
    (co-polar phi=0 plane -> |S2|^2, phi=90 plane -> |S1|^2).
    """
    m = np.sqrt(np.conj(complex(eps_r)))
    x = k_bg * radius
    theta_obs = np.atleast_1d(theta_obs)
    S1, S2 = amplitudes(m, x, math.pi - theta_obs)
    return 4 * math.pi / k_bg ** 2 * (np.abs(S2) ** 2 * np.cos(phi_obs) ** 2 + np.abs(S1) ** 2 * np.sin(phi_obs) ** 2)


def near_field(eps_r: complex, radius: float, k_bg: float, points, eta: float = 376.730313668):
    """Scattered E, H (npts, 3) outside the sphere for the plane wave E = x e^{+j k z} (travelling
    along -z, unit amplitude), in this code base's e^{+j omega t} convention.

    Bohren & Huffman's series (e^{-i omega t}, incidence along +z, x-polarised):
      E_s = sum_n E_n (i a_n N_e1n - b_n M_o1n),  H_s = (1/eta) sum_n E_n (i b_n N_o1n + a_n M_e1n),
      E_n = i^n (2n + 1)/(n (n + 1)), radial function h_n^(1)(k r).
    The textbook frame is this one turned by pi about x (x' = x, y' = -y, z' = -z), and the
    e^{+j omega t} phasor is the complex conjugate of the e^{-i omega t} one (with m taken as
    sqrt(conj(eps_r)), as in bistatic_rcs)."""
    m = np.sqrt(np.conj(complex(eps_r)))
    a, b = coefficients(m, k_bg * radius)
    nmax = len(a)
    n = np.arange(1, nmax + 1)
    P = np.atleast_2d(np.asarray(points, dtype=np.float64))
    Pp = P * np.array([1.0, -1.0, -1.0])
    r = np.linalg.norm(Pp, axis=1)
    th = np.arccos(np.clip(Pp[:, 2] / r, -1.0, 1.0))
    ph = np.arctan2(Pp[:, 1], Pp[:, 0])
    rho = k_bg * r
    pi_n, tau_n = angular(nmax, th)                                     # (nmax, npts)
    jn = special.spherical_jn(n[:, None], rho[None, :])
    yn = special.spherical_yn(n[:, None], rho[None, :])
    djn = special.spherical_jn(n[:, None], rho[None, :], derivative=True)
    dyn = special.spherical_yn(n[:, None], rho[None, :], derivative=True)
    z = jn + 1j * yn                                                    # h_n^(1)
    dz = (z + rho[None, :] * (djn + 1j * dyn)) / rho[None, :]           # (rho h_n)' / rho
    En = (1j ** n * (2 * n + 1) / (n * (n + 1)))[:, None]
    cp, sp, st = np.cos(ph)[None, :], np.sin(ph)[None, :], np.sin(th)[None, :]
    nn1 = (n * (n + 1))[:, None]
    # N_e1n, M_o1n, N_o1n, M_e1n as (r, theta, phi) components
    Ne = (cp * nn1 * st * pi_n * z / rho[None, :], cp * tau_n * dz, -sp * pi_n * dz)
    Mo = (0.0, cp * pi_n * z, -sp * tau_n * z)
    No = (sp * nn1 * st * pi_n * z / rho[None, :], sp * tau_n * dz, cp * pi_n * dz)
    Me = (0.0, -sp * pi_n * z, -cp * tau_n * z)
    Es = [np.sum(En * (1j * a[:, None] * Ne[c] - b[:, None] * Mo[c]), axis=0) for c in range(3)]
    Hs = [np.sum(En * (1j * b[:, None] * No[c] + a[:, None] * Me[c]), axis=0) / eta for c in range(3)]

    def cart(f):
        th_, ph_ = th, ph
        rh = np.stack([np.sin(th_) * np.cos(ph_), np.sin(th_) * np.sin(ph_), np.cos(th_)], 1)
        thh = np.stack([np.cos(th_) * np.cos(ph_), np.cos(th_) * np.sin(ph_), -np.sin(th_)], 1)
        phh = np.stack([-np.sin(ph_), np.cos(ph_), np.zeros_like(ph_)], 1)
        v = f[0][:, None] * rh + f[1][:, None] * thh + f[2][:, None] * phh
        return np.conj(v) * np.array([1.0, -1.0, -1.0])

    return cart(Es), cart(Hs)
