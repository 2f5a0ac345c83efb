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
