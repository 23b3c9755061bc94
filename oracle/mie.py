"""Mie series for a homogeneous sphere (TEST INFRASTRUCTURE).

The paper validates absorbed power against the Mie series for a plane wave on
a homogeneous dielectric sphere (Sec. V-A).  Written from the textbook form
(Bohren & Huffman 1983, ch. 4, time factor exp(-i w t), so the relative index
is m = sqrt(eps' + i sigma/(w eps0)); absorbed power does not depend on the
convention):

  a_n = (m psi_n(mx) psi_n'(x) - psi_n(x) psi_n'(mx)) / (m psi_n(mx) xi_n'(x) - xi_n(x) psi_n'(mx))
  b_n = (psi_n(mx) psi_n'(x) - m psi_n(x) psi_n'(mx)) / (psi_n(mx) xi_n'(x) - m xi_n(x) psi_n'(mx))
  C_ext = 2 pi / k^2 sum (2n+1) Re(a_n + b_n)
  C_sca = 2 pi / k^2 sum (2n+1) (|a_n|^2 + |b_n|^2)
  P_abs = (C_ext - C_sca) E0^2 / (2 eta0)

with psi_n(z) = z j_n(z), xi_n(z) = z h_n^(1)(z), x = k0 a.  Two evaluations are
provided: the logarithmic-derivative form (downward recurrence) and direct
spherical Bessel functions of complex argument; the tests compare them.
"""
import numpy as np
import scipy.special as sp

from . import physics


def _nmax(x, m):
    return int(np.ceil(max(x, abs(m) * x) + 4.0 * x ** (1.0 / 3.0) + 2.0)) + 15


def _riccati_real(n, x):
    j = sp.spherical_jn(n, x)
    jd = sp.spherical_jn(n, x, derivative=True)
    y = sp.spherical_yn(n, x)
    yd = sp.spherical_yn(n, x, derivative=True)
    psi = x * j
    dpsi = j + x * jd
    xi = x * (j + 1j * y)
    dxi = (j + 1j * y) + x * (jd + 1j * yd)
    return psi, dpsi, xi, dxi


def coefficients(x, m, method='logderiv'):
    nmax = _nmax(x, m)
    n = np.arange(1, nmax + 1)
    psi, dpsi, xi, dxi = _riccati_real(n, x)
    mx = m * x
    if method == 'logderiv':
        # D_n(mx) = psi_n'(mx)/psi_n(mx), downward: D_{n-1} = n/z - 1/(D_n + n/z)
        nstart = nmax + 30
        D = np.zeros(nstart + 1, dtype=np.complex128)
        for k in range(nstart, 0, -1):
            D[k - 1] = k / mx - 1.0 / (D[k] + k / mx)
        Dn = D[1:nmax + 1]
        psim1 = np.concatenate([[np.sin(x)], psi[:-1]])     # psi_{n-1}(x)
        xim1 = np.concatenate([[np.sin(x) - 1j * np.cos(x)], xi[:-1]])
        a = ((Dn / m + n / x) * psi - psim1) / ((Dn / m + n / x) * xi - xim1)
        b = ((m * Dn + n / x) * psi - psim1) / ((m * Dn + n / x) * xi - xim1)
    else:
        jm = sp.spherical_jn(n, mx)
        jmd = sp.spherical_jn(n, mx, derivative=True)
        psim = mx * jm
        dpsim = jm + mx * jmd
        a = (m * psim * dpsi - psi * dpsim) / (m * psim * dxi - xi * dpsim)
        b = (psim * dpsi - m * psi * dpsim) / (psim * dxi - m * xi * dpsim)
    return n, a, b


def cross_sections(radius, eps_re, sigma, freq_hz, method='logderiv'):
    k = physics.k0(freq_hz)
    m = np.sqrt(eps_re + 1j * sigma / (physics.omega(freq_hz) * physics.EPS0))
    x = k * radius
    n, a, b = coefficients(x, m, method)
    cext = 2 * np.pi / k ** 2 * np.sum((2 * n + 1) * np.real(a + b))
    csca = 2 * np.pi / k ** 2 * np.sum((2 * n + 1) * (np.abs(a) ** 2 + np.abs(b) ** 2))
    return cext, csca


def absorbed_power(radius, eps_re, sigma, freq_hz, E0=1.0, method='logderiv'):
    """Absorbed power (W) for a plane wave of amplitude E0 (V/m)."""
    cext, csca = cross_sections(radius, eps_re, sigma, freq_hz, method)
    return (cext - csca) * E0 ** 2 / (2.0 * physics.ETA0)


def coefficients_magnetic(x, m, mu_ratio):
    """a_n, b_n of a sphere with relative permeability mu_ratio = mu1 / mu
    (Bohren & Huffman eq. 4.53), direct spherical Bessel functions:
      a_n = (m psi_n(mx) psi_n'(x) - mu_ratio psi_n(x) psi_n'(mx))
            / (m psi_n(mx) xi_n'(x) - mu_ratio xi_n(x) psi_n'(mx))
      b_n = (mu_ratio psi_n(mx) psi_n'(x) - m psi_n(x) psi_n'(mx))
            / (mu_ratio psi_n(mx) xi_n'(x) - m xi_n(x) psi_n'(mx))
    with m = sqrt(eps_r mu_r) the relative index; mu_ratio = 1 gives the
    dielectric coefficients."""
    nmax = _nmax(x, m)
    n = np.arange(1, nmax + 1)
    psi, dpsi, xi, dxi = _riccati_real(n, x)
    mx = m * x
    jm = sp.spherical_jn(n, mx)
    jmd = sp.spherical_jn(n, mx, derivative=True)
    psim = mx * jm
    dpsim = jm + mx * jmd
    a = (m * psim * dpsi - mu_ratio * psi * dpsim) / (m * psim * dxi - mu_ratio * xi * dpsim)
    b = (mu_ratio * psim * dpsi - m * psi * dpsim) / (mu_ratio * psim * dxi - m * xi * dpsim)
    return n, a, b


def absorbed_power_magnetic(radius, eps_r, mu_r, freq_hz, E0=1.0):
    """Absorbed power (W) of a plane wave of amplitude E0 on a sphere of
    complex eps_r and mu_r given in the paper's convention (eq. 2, exp(+i w
    t), negative imaginary parts for loss): mapped to exp(-i w t) by
    conjugation, m = sqrt(eps mu) with a positive imaginary part."""
    k = physics.k0(freq_hz)
    e, mu = np.conj(eps_r), np.conj(mu_r)
    m = np.sqrt(e * mu)
    if m.imag < 0:
        m = -m
    n, a, b = coefficients_magnetic(k * radius, m, mu)
    cext = 2 * np.pi / k ** 2 * np.sum((2 * n + 1) * np.real(a + b))
    csca = 2 * np.pi / k ** 2 * np.sum((2 * n + 1) * (np.abs(a) ** 2 + np.abs(b) ** 2))
    return (cext - csca) * E0 ** 2 / (2.0 * physics.ETA0)
