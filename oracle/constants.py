"""Physical constants and material wavenumbers (oracle; test infrastructure only).

Time dependence e^{+j omega t}: the Green's function is e^{-jkR}/(4 pi R) (eq. hgf)
and the complex relative permittivity is eps_r - j sigma/(omega eps0) (eq. epsrc).
mu0 is taken as exactly 4 pi 1e-7 H/m (the paper does not state its constants).
"""
import cmath
import math

C0 = 299_792_458.0
MU0 = 4.0e-7 * math.pi
EPS0 = 1.0 / (MU0 * C0 * C0)
ETA0 = MU0 * C0


def omega(freq_hz: float) -> float:
    return 2.0 * math.pi * freq_hz


def k0_of(freq_hz: float) -> float:
    return omega(freq_hz) / C0


def eps_c(eps_r: complex, sigma: float, freq_hz: float) -> complex:
    """Complex relative permittivity, eq. (epsrc)."""
    return complex(eps_r) - 1j * sigma / (omega(freq_hz) * EPS0)


def wavenumber(k0: float, epsc: complex, mu_r: float) -> complex:
    """k = sqrt(eps_c mu_r) k0 on the principal branch (Im k <= 0 for lossy media)."""
    k = cmath.sqrt(complex(epsc) * mu_r) * k0
    if k.imag > 0:
        k = -k
    return k
