"""Pins of the oracle's PWC discretisation (Sec. V: 3 unknowns per voxel, 6
unique tensors), each against something other than its own formula:

* the PWC dense system equals the rows and columns a = 4 p of the PWL dense
  system (built by independent code, with its own Gram vector);
* the voxel-pair sum equals the circulant FFT route;
* the static self block of a cube, T^{pp}(0) = dV - dV / 3 at k0 = 0
  (Gram plus the depolarisation term of a cube);
* the complex symmetry of the Galerkin blocks (reciprocity), which leaves 6
  unique tensors;
* absorbed power from currents (eq. 44) equals the sum of the power density
  of the fields (1/2 sigma |e|^2 dV);
* a small sphere at low frequency: the interior field is close to the
  quasi-static 3 / (eps_r + 2) of the incident field (Clausius-Mossotti);
* the paper's comparison on a coarse sphere: the PWC absorbed power is
  farther from the Mie series than the PWL one.
"""
import functools

import numpy as np
import pytest

import vie_inputs as vi
from oracle import incident, matvec, mie, physics, post, pwc, solve, toeplitz

F = 298e6
K = physics.k0(F)


@functools.lru_cache(maxsize=None)
def _T(N, D, k0=K):
    return toeplitz.toeplitz_full(N, D, k0)


def test_dense_system_is_pwl_restricted():
    N, D = (3, 2, 2), (0.004, 0.005, 0.006)
    T = _T(N, D)
    e, s = vi.ellipsoid_phantom(N, D, 11)
    tau = physics.tau(e, s, F)
    A12 = solve.dense_prec_matrix(T, tau, D)
    NV = N[0] * N[1] * N[2]
    rows = np.concatenate([np.arange(NV) + a * NV for a in pwc.PWL_INDEX])
    A3 = pwc.dense_prec_matrix(pwc.blocks_from_pwl(T), tau, D)
    assert np.abs(A3 - A12[np.ix_(rows, rows)]).max() < 1e-14 * np.abs(A12).max()


def test_direct_sum_equals_fft_route():
    N, D = (4, 3, 5), (0.005, 0.004, 0.006)
    T3 = pwc.blocks_from_pwl(_T(N, D))
    x = vi.complex_normal(12, (3,) + N)
    y1 = pwc.direct_N(T3, x)
    for M in ((8, 6, 10), (9, 5, 12)):
        y2 = pwc.fft_N(pwc.spectrum(T3, M), x)
        assert np.abs(y2 - y1).max() < 1e-12 * np.abs(y1).max()


def test_static_self_block_of_a_cube():
    h = 0.01
    T3 = pwc.blocks_from_pwl(toeplitz.toeplitz_full((1, 1, 1), (h, h, h), 0.0))
    dv = h ** 3
    blk = T3[:, :, 0, 0, 0]
    assert np.allclose(np.diag(blk), dv * (1 - 1 / 3), rtol=1e-9, atol=0)
    off = blk - np.diag(np.diag(blk))
    assert np.abs(off).max() < 1e-9 * dv


def test_reciprocity_and_unique_tensors():
    """T(d) = T(-d)^T, and T^{pq}(d) = T^{qp}(d) for the constant functions:
    three diagonal and three off-diagonal tensors."""
    N, D = (3, 3, 2), (0.004, 0.005, 0.006)
    T3 = pwc.blocks_from_pwl(_T(N, D))
    flip = T3[:, :, ::-1, ::-1, ::-1]
    assert np.abs(T3 - flip.transpose(1, 0, 2, 3, 4)).max() < 1e-12 * np.abs(T3).max()
    assert np.abs(T3 - T3.transpose(1, 0, 2, 3, 4)).max() < 1e-12 * np.abs(T3).max()


def test_power_from_currents_equals_power_density():
    N, D = (3, 3, 3), (0.005,) * 3
    e, s = vi.ellipsoid_phantom(N, D, 13)
    chi = physics.chi(e, s, F)
    x = vi.complex_normal(14, (3,) + N) * (chi != 0)[None]
    P = pwc.absorbed_power(x, chi, D, F)
    ef = post.fields_from_currents(x, chi, F)
    assert abs(P - np.sum(pwc.power_density(ef, s)) * D[0] * D[1] * D[2]) < 1e-12 * abs(P)


def test_quasi_static_sphere_interior_field():
    N, D = (5, 5, 5), (0.002,) * 3
    f = 1e6
    e, s = vi.sphere(N, D, 0.0051, 4.0, 0.0)
    tau, chi = physics.tau(e, s, f), physics.chi(e, s, f)
    T3 = pwc.blocks_from_pwl(toeplitz.toeplitz_full(N, D, physics.k0(f)))
    et = pwc.restrict(incident.planewave_tested(N, D, physics.k0(f)))
    x = pwc.solve_dense(T3, tau, D, pwc.rhs_prec(et, tau, D, f))
    ef = post.fields_from_currents(x, chi, f)
    m = chi != 0
    ex = ef[0][m].real.mean()
    assert abs(ex - 3 / (4.0 + 2)) < 0.1 * 3 / (4.0 + 2)
    # cross components: local (staircase corners), cancelling over the
    # mirror-symmetric body
    for p in (1, 2):
        assert np.abs(ef[p][m]).max() < 0.2 * ex
        assert abs(ef[p][m].mean()) < 1e-9 * ex


def test_pwc_farther_from_mie_than_pwl():
    """Sec. V-A: on the same voxels, the PWL absorbed power is closer to the
    Mie series than the PWC one (the paper reports about 12 times)."""
    N, D = (6, 6, 6), (0.01,) * 3
    T = _T(N, D)
    e, s = vi.sphere(N, D, 0.025, 50.0, 0.7)
    tau, chi = physics.tau(e, s, F), physics.chi(e, s, F)
    et = incident.planewave_tested(N, D, K)
    x12 = solve.solve_dense(T, tau, D, matvec.rhs_prec(et, tau, D, F))
    x3 = pwc.solve_dense(pwc.blocks_from_pwl(T), tau, D, pwc.rhs_prec(pwc.restrict(et), tau, D, F))
    req = ((chi != 0).sum() * D[0] * D[1] * D[2] * 3 / (4 * np.pi)) ** (1 / 3)
    Pm = mie.absorbed_power(req, 50.0, 0.7, F)
    err12 = abs(post.absorbed_power(x12, chi, D, F) - Pm) / Pm
    err3 = abs(pwc.absorbed_power(x3, chi, D, F) - Pm) / Pm
    print("PWL %.4f PWC %.4f" % (err12, err3))
    assert err3 > 2 * err12


def test_operators_are_pwl_restricted():
    """N x, P^-1 A x and A x of the PWC system equal the PWL operators applied
    to the vector with zero linear coefficients, read at the unknowns a = 4 p."""
    N, D = (3, 4, 2), (0.005, 0.004, 0.006)
    T = _T(N, D)
    T3 = pwc.blocks_from_pwl(T)
    e, s = vi.ellipsoid_phantom(N, D, 15)
    tau, chi, er = physics.tau(e, s, F), physics.chi(e, s, F), physics.eps_r(e, s, F)
    x3 = vi.complex_normal(16, (3,) + N)
    x12 = np.zeros((12,) + N, dtype=np.complex128)
    x12[list(pwc.PWL_INDEX)] = x3
    pairs = [(pwc.direct_N(T3, x3), matvec.direct_N(T, x12)),
             (pwc.apply_prec(T3, x3, tau, D), matvec.apply_prec(T, x12, tau, D)),
             (pwc.apply_A(T3, x3, er, chi, D), matvec.apply_A(T, x12, er, chi, D))]
    for a, b in pairs:
        b3 = pwc.restrict(b)
        assert np.abs(a - b3).max() < 1e-13 * np.abs(b3).max()


def test_total_field_is_pwl_restricted():
    """The PWC total field equals the PWL one for a pulse-only current, read
    at the unknowns a = 4 p."""
    N, D = (3, 2, 4), (0.006, 0.005, 0.004)
    T = _T(N, D)
    x3 = vi.complex_normal(17, (3,) + N)
    x12 = np.zeros((12,) + N, dtype=np.complex128)
    x12[list(pwc.PWL_INDEX)] = x3
    et = incident.planewave_tested(N, D, K)
    a = pwc.total_field(pwc.blocks_from_pwl(T), x3, pwc.restrict(et), D, F)
    b = pwc.restrict(post.total_field(T, x12, et, D, F))
    assert np.abs(a - b).max() < 1e-13 * np.abs(b).max()

