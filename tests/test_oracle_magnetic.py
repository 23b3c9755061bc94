"""Pins of the oracle's magnetic operator and magnetic outputs (Sec. II eq.
8b and 'tot_fields' b, Sec. III eq. 25b, Sec. V-D): three routes to the K
blocks (reduced quadrature; power series of g with the derivative moved onto
the basis; with the derivative left on the kernel), the unreduced 6-D curl
quadrature on separated voxels, the block symmetries and the 30 unique
tensors, the static field of a uniform current in a sphere, the incident
magnetic fields against the electric ones (closed form, Ampere's law), and
hand-worked b1+ / energy / error values."""
import itertools

import numpy as np
import pytest

import vie_inputs as vi
from oracle import gaussian, incident, magnetic, matvec, physics, toeplitz, unreduced

K298 = physics.k0(298e6)
BRICK = (0.005, 0.004, 0.003)
NEAR27 = np.array(list(itertools.product((-1, 0, 1), repeat=3)))


def _blockwise_err(A, B):
    return max(float(np.abs(A[i] - B[i]).max() / np.abs(B[i]).max()) for i in range(len(B)))


def _s():
    """s(a) = prod_i sigma_i(a): -1 for the pulse, +1 for the linear functions."""
    return np.tile(np.array([-1.0, 1.0, 1.0, 1.0]), 3)


@pytest.mark.parametrize("k0", [0.0, K298])
def test_near_k_blocks_three_routes(k0):
    """All 27 touching / coincident offsets, every entry: the oracle's reduced
    quadrature, the Gaussian route with the derivative on the basis, and the
    Gaussian route with the derivative on the kernel (no face terms)."""
    A = toeplitz.galerkin_blocks(NEAR27, BRICK, k0, part='K')
    B = gaussian.blocks(NEAR27, BRICK, k0, part='K')
    C = gaussian.blocks(NEAR27, BRICK, k0, part='Kcurl')
    assert _blockwise_err(A, B) < 1e-9
    assert _blockwise_err(C, B) < 1e-9


def test_far_k_blocks_match_unreduced_6d():
    for d in [(2, 0, 0), (2, 1, 0), (0, -2, 3), (3, 2, 1)]:
        A = toeplitz.galerkin_blocks(np.array([d]), BRICK, K298, part='K')[0]
        B = unreduced.curl_block_6d(d, BRICK, K298, n=8)
        assert np.abs(A - B).max() / np.abs(B).max() < 1e-9, d


def test_k_block_symmetries_and_unique_count():
    """K(-d) = K(d)^T (curl S is symmetric under the bilinear pairing),
    reflecting axis i gives -sigma_i(a) sigma_i(b) K(d) (the curl is a
    pseudo-vector operator), K^{(p,l),(p,l')} = 0, K^{(p,l),(q,l')} =
    -K^{(q,l),(p,l')}, and 30 distinct values up to sign per offset (Sec. III-C
    counts 90 unique entries for N and K together, 60 of them N's)."""
    ds = np.concatenate([NEAR27[::2], np.array([[2, 1, 0], [3, -2, 1]])])
    Kp = toeplitz.galerkin_blocks(ds, BRICK, K298, part='K')
    scale = np.abs(Kp).max()
    Kn = toeplitz.galerkin_blocks(-ds, BRICK, K298, part='K')
    assert np.abs(Kn - Kp.transpose(0, 2, 1)).max() / scale < 1e-12
    for axis in range(3):
        dm = ds.copy()
        dm[:, axis] *= -1
        Km = toeplitz.galerkin_blocks(dm, BRICK, K298, part='K')
        r = matvec.reflection_signs(axis)
        assert np.abs(Km + np.outer(r, r)[None] * Kp).max() / scale < 1e-12
    B = Kp.reshape(-1, 3, 4, 3, 4)
    for p in range(3):
        assert not np.abs(B[:, p, :, p, :]).max()
    assert np.abs(B + B.transpose(0, 3, 2, 1, 4)).max() / scale < 1e-12
    T = toeplitz.galerkin_blocks(np.array([[3, 2, 1]]), BRICK, K298, part='K')[0]
    v = T.reshape(-1)
    v = v[np.abs(v) > 1e-14 * np.abs(T).max()]
    clusters = []
    for z in v:
        if not any(min(abs(z - c), abs(z + c)) <= 1e-9 * abs(c) for c in clusters):
            clusters.append(z)
    assert len(clusters) == 30


def test_uniform_current_in_sphere_static_field():
    """A uniform current density J x_hat in a ball gives, inside, the static
    field h = curl S J = (J x_hat x r) / 3, i.e. h_y = -z/3, h_z = y/3
    (vector potential J (3 a^2 - r^2) / 6).  The discrete G^-1 K x of a
    staircased ball at k0 -> 0 approaches it in the interior as the grid is
    refined, pulse and linear coefficients alike.  (The interior field of
    a staircased ball depends on how its surface is stepped, so the error is
    bounded rather than monotone in h; a wrong sign, axis or factor of the
    curl gives O(1) errors.)"""
    a = 0.03
    errs = []
    for n in (8, 12):
        h = 2 * a * 1.25 / n
        N, Dl = (n, n, n), (h, h, h)
        TK = toeplitz.toeplitz_full(N, Dl, 1e-6, part='K')
        cx, cy, cz = incident.voxel_centres(N, Dl)
        X, Y, Z = np.meshgrid(cx, cy, cz, indexing='ij')
        inside = X ** 2 + Y ** 2 + Z ** 2 <= a * a
        x = np.zeros((12,) + N, dtype=np.complex128)
        x[0][inside] = 1.0
        hf = magnetic.total_h(TK, x, np.zeros_like(x), Dl)
        core = X ** 2 + Y ** 2 + Z ** 2 <= (0.5 * a) ** 2
        ref_y, ref_z = -Z / 3, Y / 3
        e = max(np.abs(hf[4][core] - ref_y[core]).max(), np.abs(hf[8][core] - ref_z[core]).max()) / (a / 3)
        el = max(np.abs(hf[4 + 3][core] + h / 3).max(), np.abs(hf[8 + 2][core] - h / 3).max()) / (h / 3)
        assert np.abs(hf[0][core]).max() < 1e-3 * a / 3   # no x component
        errs.append((e, el))
    print("uniform current in a ball, interior errors (pulse, linear):", errs)
    for e, el in errs:
        assert e < 1e-2 and el < 5e-2


def test_incident_magnetic_fields():
    """The plane wave's tested h equals its tested e turned from x to y and
    divided by eta0 (closed form); the dipole's H obeys Ampere's law
    curl H = i w eps0 E away from the source (finite differences against the
    oracle's E of the same dipole)."""
    N, Dl = (3, 4, 5), (0.005, 0.004, 0.006)
    ht = magnetic.planewave_h_tested(N, Dl, K298)
    et = incident.planewave_tested(N, Dl, K298)
    ref = np.zeros_like(ht)
    ref[4:8] = et[0:4] / physics.ETA0
    assert np.abs(ht - ref).max() < 1e-12 * np.abs(ref).max()
    f = 298e6
    r0, m = np.array([0.05, -0.02, 0.01]), np.array([0.3, 0.0, 1.0])
    P = np.array([[0.01, 0.02, -0.015], [-0.03, 0.0, 0.02]])
    eps = 1e-6
    curl = np.zeros((2, 3), dtype=np.complex128)
    for k in range(3):
        dp = np.zeros(3)
        dp[k] = eps
        dH = (magnetic.dipole_h_field(P + dp, r0, m, f) - magnetic.dipole_h_field(P - dp, r0, m, f)) / (2 * eps)
        for p in range(3):
            for q in range(3):
                s = gaussian._levi(p, k, q)
                if s:
                    curl[:, p] += s * dH[:, q]
    E = incident.dipole_field(P, r0, m, f)
    rhs = 1j * physics.omega(f) * physics.EPS0 * E
    assert np.abs(curl - rhs).max() < 1e-6 * np.abs(rhs).max()


def test_b1plus_energy_and_errors_hand_computed():
    Dl = (0.002, 0.003, 0.004)
    dv = np.prod(Dl)
    h = np.zeros((12, 1, 1, 1), dtype=np.complex128)
    h[0] = 2.0          # h_x pulse
    h[4] = 1.0j         # h_y pulse
    h[5] = 3.0          # h_y linear in x
    b = magnetic.b1plus(h)
    assert b[0, 0, 0, 0] == pytest.approx(physics.MU0 * (2.0 + 1j * 1j))
    assert b[1, 0, 0, 0] == pytest.approx(physics.MU0 * 3.0j)
    w = magnetic.magnetic_energy_density(h)
    assert w[0, 0, 0] == pytest.approx(0.25 * physics.MU0 * (4.0 + 1.0 + 9.0 / 12))
    W = magnetic.magnetic_energy(h, np.ones((1, 1, 1), bool), Dl)
    assert W == pytest.approx(w[0, 0, 0] * dv)
    e1, e2, e3 = magnetic.rel_errors_h(1.2, 1.0, np.array([2.0, 1.0]), np.array([1.0, 1.0]), 2 * h, h, Dl)
    assert (e1, e2, e3) == pytest.approx((0.2, 0.5, 1.0))
