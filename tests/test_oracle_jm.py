"""Pins of the oracle's J-M formulation (Sec. II eq. 13-15: polarisation
and magnetisation currents, magnetic contrast) and of the Mie series with a
permeable sphere:

* Mie with mu_r = 1 is the dielectric series; exchanging eps_r and mu_r
  leaves the absorbed power unchanged (duality); a lossless sphere absorbs
  nothing;
* without magnetic contrast the J-M solution is the dielectric one with
  x_m = 0; without electric contrast x_j = 0 and x_m solves the dielectric
  system with (mu, h, c_m) in place of (eps, e, c_e);
* reciprocity: diag((c_e chi_e)^-1, -(c_m chi_m)^-1) A is complex
  symmetric (the Galerkin matrices of N and K are both symmetric), which
  fixes the signs and constants of the coupling blocks;
* a small permeable sphere has the quasi-static interior field
  3 / (mu_r + 2) H0;
* a magneto-dielectric sphere absorbs the Mie power within the coarse
  grid's discretisation error (3.4% at 6^3, against 3.5x for a sphere
  without its permeability).
"""
import numpy as np

import vie_inputs as vi
from oracle import incident, jm, magnetic, matvec, mie, physics, solve, toeplitz

F = 298e6
K = physics.k0(F)


def _materials(e, s, mur, f=F):
    er = physics.eps_r(e, s, f)
    chie, chim = er - 1, mur - 1
    return er, chie, chim, chie / er, chim / mur


def test_mie_magnetic_reduces_and_duality():
    a = 0.03
    for eps_re, sigma in ((50.0, 0.7), (5.0, 0.0)):
        er = physics.eps_r(eps_re, sigma, F)
        P1 = mie.absorbed_power(a, eps_re, sigma, F)
        P2 = mie.absorbed_power_magnetic(a, er, 1.0 + 0j, F)
        assert abs(P1 - P2) <= 1e-10 * max(abs(P1), 1e-30) + 1e-25
    er, mr = 20.0 - 4.0j, 3.0 - 1.0j
    Pa = mie.absorbed_power_magnetic(a, er, mr, F)
    Pb = mie.absorbed_power_magnetic(a, mr, er, F)
    assert Pa > 0 and abs(Pa - Pb) / Pa < 1e-10
    k = physics.k0(F)
    n, A, B = mie.coefficients_magnetic(k * a, np.sqrt(20.0 * 3.0 + 0j), 3.0)
    cext = np.sum((2 * n + 1) * np.real(A + B))
    csca = np.sum((2 * n + 1) * (np.abs(A) ** 2 + np.abs(B) ** 2))
    assert abs(cext - csca) < 1e-10 * cext                 # lossless


def test_without_magnetic_contrast_is_the_dielectric_solution():
    N, D = (3, 2, 2), (0.006, 0.005, 0.004)
    TN, TK = toeplitz.toeplitz_full(N, D, K), toeplitz.toeplitz_full(N, D, K, part='K')
    e, s = vi.ellipsoid_phantom(N, D, 5)
    er, chie, chim, taue, taum = _materials(e, s, np.ones(N, dtype=np.complex128))
    et = incident.planewave_tested(N, D, K)
    ht = magnetic.planewave_h_tested(N, D, K)
    x = jm.solve_dense(TN, TK, taue, taum, D, F, jm.rhs_prec(et, ht, taue, taum, D, F))
    xd = solve.solve_dense(TN, taue, D, matvec.rhs_prec(et, taue, D, F))
    assert np.abs(x[12:]).max() <= 1e-13 * np.abs(x).max()      # zero up to the LU's rounding
    assert np.abs(x[:12] - xd).max() < 1e-12 * np.abs(xd).max()


def test_without_electric_contrast_is_the_dual_system():
    N, D = (2, 3, 2), (0.005, 0.004, 0.006)
    TN, TK = toeplitz.toeplitz_full(N, D, K), toeplitz.toeplitz_full(N, D, K, part='K')
    rng = np.random.default_rng(3)
    mur = 1.0 + rng.uniform(0.5, 4.0, N) - 1j * rng.uniform(0.0, 1.0, N)
    er, chie, chim, taue, taum = _materials(np.ones(N), np.zeros(N), mur)
    et = incident.planewave_tested(N, D, K)
    ht = magnetic.planewave_h_tested(N, D, K)
    x = jm.solve_dense(TN, TK, taue, taum, D, F, jm.rhs_prec(et, ht, taue, taum, D, F))
    assert np.abs(x[:12]).max() <= 1e-13 * np.abs(x).max()
    G = physics.gram_vector(*D)[:, None, None, None]
    xm = solve.solve_dense(TN, taum, D, physics.c_m(F) * taum * ht / G)
    assert np.abs(x[12:] - xm).max() < 1e-12 * np.abs(xm).max()


def test_reciprocity_of_the_scaled_operator():
    """u^T D A v = v^T D A u with D = diag((c_e chi_e)^-1, -(c_m chi_m)^-1):
    the Galerkin matrices of N and of K = curl S are both symmetric (the
    curl moves across the bilinear form and commutes with S), so the
    scaled operator [[(eps G - chi_e N)/(c_e chi_e), K], [K, -(mu G -
    chi_m N)/(c_m chi_m)]] is.  The other sign of the second row breaks it
    by the size of the coupling, which pins the coupling constants."""
    N, D = (3, 2, 3), (0.005, 0.004, 0.006)
    TN, TK = toeplitz.toeplitz_full(N, D, K), toeplitz.toeplitz_full(N, D, K, part='K')
    rng = np.random.default_rng(7)
    e = rng.uniform(2.0, 60.0, N)
    s = rng.uniform(0.0, 1.5, N)
    mur = rng.uniform(1.5, 4.0, N) - 1j * rng.uniform(0.0, 1.0, N)
    er, chie, chim, taue, taum = _materials(e, s, mur)
    u = vi.complex_normal(11, (24,) + N)
    v = vi.complex_normal(12, (24,) + N)
    asym = {}
    for sgn in (-1.0, 1.0):
        Dsc = np.concatenate([np.broadcast_to(1.0 / (physics.c_e(F) * chie), (12,) + N),
                              np.broadcast_to(sgn / (physics.c_m(F) * chim), (12,) + N)])
        lhs = np.sum(u * Dsc * jm.apply_A(TN, TK, v, er, chie, mur, chim, D, F))
        rhs = np.sum(v * Dsc * jm.apply_A(TN, TK, u, er, chie, mur, chim, D, F))
        asym[sgn] = abs(lhs - rhs) / abs(lhs)
    assert asym[-1.0] < 1e-12
    assert asym[1.0] > 1e-7


def test_quasi_static_permeable_sphere():
    """Electrically small sphere, mu_r = 4 without electric contrast: the
    interior magnetic field is close to 3/(mu_r + 2) H0 = 0.5 H0."""
    N, D = (6, 6, 6), (0.004,) * 3
    f = 10e6
    k = physics.k0(f)
    TN, TK = toeplitz.toeplitz_full(N, D, k), toeplitz.toeplitz_full(N, D, k, part='K')
    e, s = vi.sphere(N, D, 0.0121, 4.0, 0.0)
    inside = e != 1.0
    mur = np.where(inside, 4.0 + 0j, 1.0 + 0j)
    er, chie, chim, taue, taum = _materials(np.ones(N), np.zeros(N), mur, f)
    et = incident.planewave_tested(N, D, k)
    ht = magnetic.planewave_h_tested(N, D, k)
    b = jm.rhs_prec(et, ht, taue, taum, D, f)
    x, info = solve.gmres(lambda v: jm.apply_prec(TN, TK, v, taue, taum, D, f), b, restart=50, tol=1e-10)
    assert info["converged"]
    hf = jm.fields(x, chie, chim, f)[12:]
    hy = hf[4][inside] * physics.ETA0                      # pulse coefficient of h_y, H0 = 1 / eta0
    assert abs(np.mean(hy.real) - 0.5) < 0.05
    assert np.abs(hy.imag).max() < 0.01


def test_magnetodielectric_sphere_absorbs_mie_power():
    N, h = (6, 6, 6), 0.01
    Dl = (h,) * 3
    TN, TK = toeplitz.toeplitz_full(N, Dl, K), toeplitz.toeplitz_full(N, Dl, K, part='K')
    M = tuple(2 * n for n in N)
    CN, CK = matvec.circulant_spectrum(TN, M), matvec.circulant_spectrum(TK, M)
    e, s = vi.sphere(N, Dl, 0.025, 50.0, 0.7)
    inside = e != 1.0
    mu_in = 2.0 - 0.5j
    er, chie, chim, taue, taum = _materials(e, s, np.where(inside, mu_in, 1.0 + 0j))
    b = jm.rhs_prec(incident.planewave_tested(N, Dl, K), magnetic.planewave_h_tested(N, Dl, K), taue, taum, Dl, F)
    x, info = solve.gmres(lambda v: jm.apply_prec(CN, CK, v, taue, taum, Dl, F, Nx_fn=matvec.fft_N,
                                                 Kx_fn=matvec.fft_N), b, restart=50, tol=1e-8)
    assert info["converged"]
    P = jm.absorbed_power(x, chie, chim, Dl, F)
    req = (inside.sum() * h ** 3 * 3 / (4 * np.pi)) ** (1 / 3)
    Pm = mie.absorbed_power_magnetic(req, er[inside][0], mu_in, F)
    assert abs(P - Pm) / Pm < 0.06
    assert Pm > 3 * mie.absorbed_power(req, 50.0, 0.7, F)   # the permeability matters
