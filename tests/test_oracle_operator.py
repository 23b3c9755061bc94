"""Pins of the oracle's operator products, right-hand sides, solves, post
processing and Mie series."""
import functools

import numpy as np
import pytest

import vie_inputs as vi
from oracle import incident, matvec, mie, physics, post, solve, toeplitz

F = 298e6
K = physics.k0(F)
D = (0.006, 0.005, 0.007)


@functools.lru_cache(None)
def _blocks(N, Delta=D, k0=K):
    return toeplitz.toeplitz_full(N, Delta, k0)


def test_direct_sum_matches_brute_force_pairs():
    """direct_N regroups sum_n T(m - n) x_n by offset; check against the
    double loop over voxel pairs on a 2x3x2 grid with random blocks."""
    N = (2, 3, 2)
    T = vi.complex_normal(1, (12, 12, 3, 5, 3))
    x = vi.complex_normal(2, (12,) + N)
    y = np.zeros_like(x)
    for m in np.ndindex(*N):
        for n in np.ndindex(*N):
            d = [m[i] - n[i] + N[i] - 1 for i in range(3)]
            y[(slice(None),) + m] += T[:, :, d[0], d[1], d[2]] @ x[(slice(None),) + n]
    assert np.abs(matvec.direct_N(T, x) - y).max() < 1e-12


@pytest.mark.parametrize("M", [(6, 8, 4), (5, 7, 3), (12, 9, 10)])
def test_fft_product_equals_direct_sum(M):
    """Circulant embedding + FFT reproduces the Toeplitz product exactly for any
    M_i >= 2 N_i - 1 (Sec. IV-A), random blocks."""
    N = (3, 4, 2)
    T = vi.complex_normal(3, (12, 12, 5, 7, 3))
    x = vi.complex_normal(4, (12,) + N)
    y = matvec.fft_N(matvec.circulant_spectrum(T, M), x)
    assert np.abs(y - matvec.direct_N(T, x)).max() / np.abs(y).max() < 1e-13


def test_full_from_octant_matches_direct_blocks():
    N = (3, 2, 3)
    Tf = _blocks(N)
    Toct = Tf[:, :, N[0] - 1:, N[1] - 1:, N[2] - 1:]
    assert np.abs(matvec.full_from_octant(Toct) - Tf).max() / np.abs(Tf).max() < 1e-12


def test_spectrum_fold_signs():
    """With M = 2N (middle index zero), the circulant spectrum satisfies
    C^ab(.., M_i - xi_i, ..) = sigma_i(a) sigma_i(b) C^ab(.., xi_i, ..), so the
    octant xi_i <= M_i/2 determines it."""
    N = (3, 2, 3)
    M = (6, 4, 6)
    Ch = matvec.circulant_spectrum(_blocks(N), M)
    for axis in range(3):
        r = matvec.reflection_signs(axis)
        flipped = np.roll(np.flip(Ch, axis=2 + axis), 1, axis=2 + axis)   # index M - xi
        sgn = np.outer(r, r)[:, :, None, None, None]
        assert np.abs(flipped - sgn * Ch).max() / np.abs(Ch).max() < 1e-12


def test_planewave_closed_form_vs_quadrature():
    N = (3, 2, 5)
    a = incident.planewave_tested(N, D, K)
    b = incident.tested_by_quadrature(lambda P: incident.planewave_field(P, K), N, D, nq=8)
    assert np.abs(a - b).max() / np.abs(a).max() < 1e-14
    # high k: the closed form still matches (checks the l=4 formula)
    a = incident.planewave_tested(N, D, 300.0)
    b = incident.tested_by_quadrature(lambda P: incident.planewave_field(P, 300.0), N, D, nq=12)
    assert np.abs(a - b).max() / np.abs(a).max() < 1e-13


def test_dipole_field_solves_helmholtz_and_static_limit():
    """curl curl E - k0^2 E = 0 away from the source (finite differences), and
    near the source E -> p (3 (R.u)R - u) / (4 pi eps0 R^3) with p = I l/(i w)."""
    r0 = np.array([0.01, -0.02, 0.03])
    m = np.array([0.3, -0.5, 0.8])
    P0 = np.array([0.11, 0.05, -0.07])
    h = 1e-4

    def E(P):
        return incident.dipole_field(np.asarray(P)[None], r0, m, F)[0]

    def jac(fn, P):
        return np.stack([(fn(P + h * e) - fn(P - h * e)) / (2 * h) for e in np.eye(3)], 1)

    def curl(fn):
        def c(P):
            J = jac(fn, P)
            return np.array([J[2, 1] - J[1, 2], J[0, 2] - J[2, 0], J[1, 0] - J[0, 1]])
        return c
    cc = curl(curl(E))(P0)
    resid = cc - K ** 2 * E(P0)
    assert np.abs(resid).max() / (K ** 2 * np.abs(E(P0)).max()) < 1e-3
    Rv = np.array([1e-4, 2e-4, -1.5e-4])
    R = np.linalg.norm(Rv)
    Rh = Rv / R
    p = m / (1j * physics.omega(F))
    stat = (3 * Rh * (Rh @ p) - p) / (4 * np.pi * physics.EPS0 * R ** 3)
    assert np.abs(E(r0 + Rv) - stat).max() / np.abs(stat).max() < 1e-5   # O((k R)^2)


def test_gmres_matches_dense_solve():
    N = (3, 3, 3)
    T = _blocks(N)
    e, s = vi.sphere(N, D, 0.008, 50.0, 0.7)
    tau = physics.tau(e, s, F)
    b = matvec.rhs_prec(incident.planewave_tested(N, D, K), tau, D, F)
    xd = solve.solve_dense(T, tau, D, b)
    x, info = solve.gmres(lambda v: matvec.apply_prec(T, v, tau, D), b, restart=10, tol=1e-12)
    assert info['converged']
    assert np.abs(x - xd).max() / np.abs(xd).max() < 1e-10


def test_preconditioned_and_plain_operator_agree():
    """P^-1 (A x) with P = M_eps G equals the preconditioned product (eq. 17)."""
    N = (3, 2, 2)
    T = _blocks(N)
    e, s = vi.ellipsoid_phantom(N, D, 7)
    er, ch, ta = physics.eps_r(e, s, F), physics.chi(e, s, F), physics.tau(e, s, F)
    x = vi.complex_normal(5, (12,) + N)
    G = physics.gram_vector(*D)[:, None, None, None]
    Ax = matvec.apply_A(T, x, er, ch, D)
    assert np.abs(Ax / (er[None] * G) - matvec.apply_prec(T, x, ta, D)).max() < 1e-10 * np.abs(x).max()


def test_zero_contrast_is_identity():
    N = (2, 2, 2)
    T = _blocks(N)
    x = vi.complex_normal(6, (12,) + N)
    assert np.abs(matvec.apply_prec(T, x, np.zeros(N), D) - x).max() == 0.0
    _, info = solve.gmres(lambda v: v, x, tol=1e-12)
    assert info['iters'] == 1


def test_quasi_static_sphere_internal_field():
    """Electrically small sphere: the internal field is close to uniform
    3/(eps_r + 2) E0 (Clausius-Mossotti), up to staircasing.  A missing
    identity part of N or a sign error in the charge terms fails this."""
    N = (6, 6, 6)
    Dl = (0.004, 0.004, 0.004)
    f = 10e6
    k = physics.k0(f)
    T = toeplitz.toeplitz_full(N, Dl, k)
    e, s = vi.sphere(N, Dl, 0.0121, 4.0, 0.0)
    tau, chi = physics.tau(e, s, f), physics.chi(e, s, f)
    b = matvec.rhs_prec(incident.planewave_tested(N, Dl, k), tau, Dl, f)
    x = solve.solve_dense(T, tau, Dl, b)
    ef = post.fields_from_currents(x, chi, f)
    inside = chi != 0
    ex = ef[0][inside]
    assert abs(np.mean(ex.real) - 0.5) < 0.05          # 136 voxels: staircase
    assert np.abs(ex.imag).max() < 0.01
    assert np.abs(ef[4][inside]).max() < 0.25 * np.abs(ex).max()


def test_post_power_identities():
    N = (3, 3, 3)
    T = _blocks(N)
    e, s = vi.sphere(N, D, 0.01, 50.0, 0.7)
    tau, chi = physics.tau(e, s, F), physics.chi(e, s, F)
    et = incident.planewave_tested(N, D, K)
    b = matvec.rhs_prec(et, tau, D, F)
    x = solve.solve_dense(T, tau, D, b)
    P = post.absorbed_power(x, chi, D, F)
    ef = post.fields_from_currents(x, chi, F)
    p = post.power_density(ef, s)
    assert P > 0
    assert abs(P - p.sum() * np.prod(D)) / P < 1e-12
    # the field from one operator product (Sec. IV-C) equals x / (c_e chi)
    et_full = post.total_field(T, x, et, D, F)
    inside = chi != 0
    assert np.abs(et_full[:, inside] - ef[:, inside]).max() / np.abs(ef).max() < 1e-9
    # lossless material absorbs nothing
    tau0, chi0 = physics.tau(e, 0 * s, F), physics.chi(e, 0 * s, F)
    x0 = solve.solve_dense(T, tau0, D, matvec.rhs_prec(et, tau0, D, F))
    assert abs(post.absorbed_power(x0, chi0, D, F)) < 1e-12 * P


def test_mie_two_evaluations_agree_and_limits():
    for (r, e, s, f) in [(0.03, 50.0, 0.7, 298e6), (0.075, 64.0, 0.51, 298.06e6), (0.075, 227.0, 0.25, 21.29e6)]:
        a = mie.absorbed_power(r, e, s, f)
        b = mie.absorbed_power(r, e, s, f, method='bessel')
        assert abs(a - b) / a < 1e-10
    # lossless: extinction = scattering (optical theorem)
    ce, cs = mie.cross_sections(0.05, 20.0, 0.0, 298e6)
    assert abs(ce - cs) / cs < 1e-10
    # Rayleigh limit: C_abs = 4 pi k a^3 Im((m^2-1)/(m^2+2)) for k a, |m| k a << 1
    r, e, s, f = 0.001, 10.0, 0.5, 50e6
    k = physics.k0(f)
    m2 = e + 1j * s / (physics.omega(f) * physics.EPS0)
    ray = 4 * np.pi * k * r ** 3 * np.imag((m2 - 1) / (m2 + 2))
    ce, cs = mie.cross_sections(r, e, s, f)
    assert abs((ce - cs) - ray) / ray < 1e-3


def test_vie_absorbed_power_near_mie():
    """Trend check only (parity unpinned: the paper's error curves are in a
    figure that is not available): a coarse PWL sphere (6^3 voxels of 1 cm)
    is within 15% of Mie for the volume-equivalent radius (it is 10.7% off)."""
    N = (6, 6, 6)
    h = 0.01
    Dl = (h, h, h)
    T = toeplitz.toeplitz_full(N, Dl, K)
    e, s = vi.sphere(N, Dl, 0.025, 50.0, 0.7)
    tau, chi = physics.tau(e, s, F), physics.chi(e, s, F)
    x = solve.solve_dense(T, tau, Dl, matvec.rhs_prec(incident.planewave_tested(N, Dl, K), tau, Dl, F))
    P = post.absorbed_power(x, chi, Dl, F)
    req = ((chi != 0).sum() * h ** 3 * 3 / (4 * np.pi)) ** (1 / 3)
    Pm = mie.absorbed_power(req, 50.0, 0.7, F)
    assert abs(P - Pm) / Pm < 0.15


def test_unpreconditioned_rhs_gives_the_same_solution():
    """b = c_e chi e_t (eq. 31) with A x = b (eq. 24, dense from apply_A
    column by column) has the solution of the preconditioned system
    P^-1 A x = P^-1 b solved with rhs_prec: a dropped c_e, chi or Gram factor
    in either right-hand side, or in A, breaks the equality."""
    N, Dl = (2, 2, 2), (0.006, 0.005, 0.004)
    T = _blocks(N, Dl)
    e, s = vi.ellipsoid_phantom(N, Dl, 41)
    e[0, 0, 0], s[0, 0, 0] = 1.0, 0.0          # one air voxel: chi = 0 there
    er, ch, ta = physics.eps_r(e, s, F), physics.chi(e, s, F), physics.tau(e, s, F)
    et = incident.planewave_tested(N, Dl, K)
    n = 12 * np.prod(N)
    A = np.zeros((n, n), dtype=np.complex128)
    for j in range(n):
        u = np.zeros(n, dtype=np.complex128)
        u[j] = 1.0
        A[:, j] = matvec.apply_A(T, u.reshape((12,) + N), er, ch, Dl).reshape(-1)
    x_a = np.linalg.solve(A, matvec.rhs(et, ch, F).reshape(-1)).reshape((12,) + N)
    x_p = solve.solve_dense(T, ta, Dl, matvec.rhs_prec(et, ta, Dl, F))
    assert np.abs(x_a - x_p).max() < 1e-10 * np.abs(x_p).max()
    assert np.abs(x_a[:, 0, 0, 0]).max() < 1e-12 * np.abs(x_p).max()   # no current where chi = 0


def test_error_metrics_hand_computed():
    """error_e1..e3 of Sec. V-C on values worked out by hand, and error_e3
    as the relative L2 norm of the field itself: the Gram weights (eq. 33)
    against Gauss quadrature of sum_l e^{pl} N^l over the voxel."""
    Dl = (0.002, 0.003, 0.004)
    dv = np.prod(Dl)
    e_ref = np.ones((12, 1, 1, 1), dtype=np.complex128)
    e = e_ref.copy()
    e[0] = 2.0                                  # pulse of the x component off by 1
    p_ref = np.array([1.0, 1.0])
    p = np.array([1.0, 2.0])
    e1, e2, e3 = post.rel_errors(1.1, 1.0, p, p_ref, e, e_ref, Dl)
    assert e1 == pytest.approx(0.1, rel=1e-14)
    assert e2 == pytest.approx(0.5, rel=1e-14)
    # |e - e_ref|^2 weighted: dV; |e_ref|^2 weighted: 3 dV (1 + 3 / 12)
    assert e3 == pytest.approx(np.sqrt(1.0 / 3.75), rel=1e-14)
    # the weighted norm is the L2 norm of the field sum_l e^{pl} N^l(r)
    g = vi.rng(5)
    a = g.normal(size=(12, 1, 1, 1)) + 1j * g.normal(size=(12, 1, 1, 1))
    b = g.normal(size=(12, 1, 1, 1)) + 1j * g.normal(size=(12, 1, 1, 1))
    x, w = np.polynomial.legendre.leggauss(4)
    pts = [0.5 * Dl[i] * x for i in range(3)]
    wts = [0.5 * Dl[i] * w for i in range(3)]
    X, Y, Z = np.meshgrid(*pts, indexing='ij')
    W = np.einsum('i,j,k->ijk', *wts)
    basis = [np.ones_like(X), X / Dl[0], Y / Dl[1], Z / Dl[2]]

    def l2(c):
        tot = 0.0
        for pc in range(3):
            f = sum(c[4 * pc + l, 0, 0, 0] * basis[l] for l in range(4))
            tot += np.sum(W * np.abs(f) ** 2)
        return tot
    _, _, e3q = post.rel_errors(1.0, 1.0, p_ref, p_ref, a, b, Dl)
    assert e3q == pytest.approx(np.sqrt(l2(a - b) / l2(b)), rel=1e-12)
    assert l2(b) == pytest.approx(np.sum(np.abs(b[:, 0, 0, 0]) ** 2 * np.tile([1, 1 / 12, 1 / 12, 1 / 12], 3)) * dv,
                                  rel=1e-12)
