"""Physical constants and material maps (TEST INFRASTRUCTURE, see package doc).

Paper: Sec. II, eq. (1)-(2) (complex relative permittivity and permeability
with time factor exp(+i w t)), eq. (6)-(7) (c_e = i w eps0, c_m = i w mu0,
chi = eps_r - 1, chi_m = mu_r - 1), Sec. IV-B (tau = chi / eps_r).
"""
import numpy as np

# CODATA 2018
EPS0 = 8.8541878128e-12
MU0 = 1.25663706212e-6
C0 = 1.0 / np.sqrt(MU0 * EPS0)
ETA0 = np.sqrt(MU0 / EPS0)


def omega(freq_hz):
    return 2.0 * np.pi * freq_hz


def k0(freq_hz):
    """Free-space wavenumber k0 = w sqrt(mu0 eps0) (Sec. II, after eq. 2)."""
    return omega(freq_hz) * np.sqrt(MU0 * EPS0)


def c_e(freq_hz):
    """c_e = i w eps0 (eq. 6)."""
    return 1j * omega(freq_hz) * EPS0


def c_m(freq_hz):
    """c_m = i w mu0 (eq. 6)."""
    return 1j * omega(freq_hz) * MU0


def mu_r(mu_re, mu_im):
    """mu_r = mu' - i mu'' (eq. 2, time factor exp(+i w t))."""
    return np.asarray(mu_re, dtype=np.float64) - 1j * np.asarray(mu_im, dtype=np.float64)


def eps_r(eps_re, sigma, freq_hz):
    """eps_r = eps' - i eps'' with eps'' = sigma / (w eps0) (eq. 2, time
    factor exp(+i w t))."""
    return np.asarray(eps_re, dtype=np.float64) - 1j * np.asarray(sigma, dtype=np.float64) / (omega(freq_hz) * EPS0)


def chi(eps_re, sigma, freq_hz):
    """Electric susceptibility chi_e = eps_r - 1 (eq. 7)."""
    return eps_r(eps_re, sigma, freq_hz) - 1.0


def tau(eps_re, sigma, freq_hz):
    """tau_e = chi_e / eps_r (Sec. IV-B, eq. 17)."""
    er = eps_r(eps_re, sigma, freq_hz)
    return (er - 1.0) / er


def gram_diag(dx, dy, dz):
    """Diagonal of the Gram matrix per scalar basis l = 1..4 (eq. 33):
    dV for the pulse, dV/12 for the three linear functions."""
    dv = dx * dy * dz
    return np.array([dv, dv / 12.0, dv / 12.0, dv / 12.0])


def gram_vector(dx, dy, dz):
    """Gram diagonal for the 12 unknowns of a voxel, ordered a = 4 p + (l - 1)
    with p in (x, y, z) and l in 1..4 (eq. 30 ordering x^{pl})."""
    return np.tile(gram_diag(dx, dy, dz), 3)
