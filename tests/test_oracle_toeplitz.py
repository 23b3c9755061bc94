"""Pins of the oracle's Galerkin blocks (Sec. III-B/C, eq. 25a, 33, 42-43)
against things other than itself: a closed-form static potential, brute-force
6-D quadrature, differential identities and symmetries."""
import numpy as np
import pytest

from oracle import matvec, physics, toeplitz, unreduced

F298 = 298e6
K298 = physics.k0(F298)
CUBE = (0.005, 0.005, 0.005)
BRICK = (0.005, 0.004, 0.006)
NEAR = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 0], [1, 0, 1],
                 [0, 1, 1], [1, 1, 1], [-1, 0, 0], [1, -1, 0], [-1, 1, -1]])
MID = np.array([[2, 0, 0], [2, 1, 0], [0, -2, 1], [3, 2, 1], [-4, 1, 2]])


def _box_potential(P, lo, hi):
    """Closed-form int_box dr'/|P - r'| of a uniform rectangular box: sum over
    the 8 corners of the triple antiderivative
    F = xy ln(z+R) + yz ln(x+R) + zx ln(y+R)
        - x^2/2 atan(yz/(xR)) - y^2/2 atan(zx/(yR)) - z^2/2 atan(xy/(zR))."""
    def F(x, y, z):
        R = np.sqrt(x * x + y * y + z * z)
        with np.errstate(divide='ignore', invalid='ignore'):
            return (x * y * np.log(z + R) + y * z * np.log(x + R) + z * x * np.log(y + R)
                    - 0.5 * x * x * np.arctan(y * z / (x * R)) - 0.5 * y * y * np.arctan(z * x / (y * R))
                    - 0.5 * z * z * np.arctan(x * y / (z * R)))
    tot = 0.0
    for i, xx in enumerate([lo[0], hi[0]]):
        for j, yy in enumerate([lo[1], hi[1]]):
            for k, zz in enumerate([lo[2], hi[2]]):
                tot = tot + (-1) ** (i + j + k + 1) * F(xx - P[..., 0], yy - P[..., 1], zz - P[..., 2])
    return tot


def _gauss_box(n, lo, hi):
    x, w = np.polynomial.legendre.leggauss(n)
    pts = [lo[i] + (hi[i] - lo[i]) * 0.5 * (x + 1) for i in range(3)]
    wts = [(hi[i] - lo[i]) * 0.5 * w for i in range(3)]
    X = np.stack(np.meshgrid(*pts, indexing='ij'), -1).reshape(-1, 3)
    W = np.einsum('i,j,k->ijk', *wts).reshape(-1)
    return X, W


def test_box_potential_formula_far_point():
    # the closed form itself against plain quadrature where 1/r is smooth
    X, W = _gauss_box(24, (0, 0, 0), (1, 1, 1))
    P = np.array([2.3, 0.4, -1.1])
    assert abs(_box_potential(P, (0, 0, 0), (1, 1, 1)) - np.sum(W / np.linalg.norm(X - P, axis=1))) < 1e-13


@pytest.mark.parametrize("Delta", [(1.0, 1.0, 1.0), (1.0, 0.8, 1.3)])
def test_static_scalar_block_matches_closed_form(Delta):
    """S^{11}(d) at k0 = 0 equals (1/4pi) int_{V_m} phi_n, phi_n the closed-form
    box potential; covers the coincident, face-, edge- and corner-touching
    voxels where the oracle uses its singular (Duffy) quadrature."""
    ds = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 0], [1, 1, 1], [2, 1, 0]])
    S = toeplitz.galerkin_blocks(ds, Delta, 0.0, part='S')
    D = np.array(Delta)
    for i, d in enumerate(ds):
        lo_m = d * D - D / 2
        X, W = _gauss_box(48, lo_m, lo_m + D)
        ref = np.sum(W * _box_potential(X, -D / 2, D / 2)) / (4 * np.pi)
        assert abs(S[i, 0, 0] - ref) / ref < 1e-9, (d, S[i, 0, 0], ref)
        assert abs(S[i, 0, 0].imag) < 1e-20


def test_static_self_term_cube():
    """For a cube at k0 = 0, by cubic symmetry and the trace identity,
    L^{p1,p1}(0) = -dV/3, i.e. N^{p1,p1}(0) = 2 dV / 3."""
    T = toeplitz.galerkin_blocks(np.array([[0, 0, 0]]), CUBE, 0.0)[0]
    dv = np.prod(CUBE)
    for p in range(3):
        assert abs(T[4 * p, 4 * p] - 2 * dv / 3) / dv < 1e-12


@pytest.mark.parametrize("Delta,k0", [(CUBE, K298), (BRICK, K298), (BRICK, 80.0)])
def test_trace_identity(Delta, k0):
    """sum_p C^{pl,pl'}(d) = k0^2 S^{ll'}(d) + delta_{d0} delta_{ll'} G^l, from
    sum_p d_p d_p = Laplacian and (Laplacian + k0^2) g = -delta (eq. 10);
    holds at every offset, including the singular ones."""
    ds = np.concatenate([NEAR, MID])
    C = toeplitz.galerkin_blocks(ds, Delta, k0, part='C')
    S = toeplitz.galerkin_blocks(ds, Delta, k0, part='S')
    G = physics.gram_diag(*Delta)
    for i, d in enumerate(ds):
        tr = sum(C[i][4 * p:4 * p + 4, 4 * p:4 * p + 4] for p in range(3))
        rhs = k0 ** 2 * S[i] + (np.diag(G) if not d.any() else 0)
        scale = np.abs(C[i]).max()
        assert np.abs(tr - rhs).max() / scale < 1e-11, d


def test_dyadic_and_basis_swap_symmetries():
    """T^{(p,l),(q,l')} = T^{(q,l),(p,l')} (the dyadic kernel is symmetric) and
    T^{(p,l'),(q,l)} = s(l)s(l') T^{(p,l),(q,l')} with s = +1 for the pulse,
    -1 for the odd linear functions; the charge form computes each side from
    different face/volume terms, so these are non-trivial."""
    ds = np.concatenate([NEAR, MID])
    T = toeplitz.galerkin_blocks(ds, BRICK, K298).reshape(-1, 3, 4, 3, 4)
    s = np.array([1.0, -1.0, -1.0, -1.0])
    for i in range(len(ds)):
        B = T[i]
        scale = np.abs(B).max()
        assert np.abs(B - B.transpose(2, 1, 0, 3)).max() / scale < 1e-12
        assert np.abs(B.transpose(0, 3, 2, 1) - s[None, :, None, None] * s[None, None, None, :] * B).max() / scale < 1e-12


def test_reflection_and_reciprocity():
    """T(.., -d_i, ..) = sigma_i(a) sigma_i(b) T(d) and T(-d) = T(d)^T."""
    ds = np.concatenate([NEAR[:8], MID[:3]])
    Tp = toeplitz.galerkin_blocks(ds, BRICK, K298)
    for axis in range(3):
        dm = ds.copy()
        dm[:, axis] *= -1
        Tm = toeplitz.galerkin_blocks(dm, BRICK, K298)
        r = matvec.reflection_signs(axis)
        err = np.abs(Tm - np.outer(r, r)[None] * Tp).max() / np.abs(Tp).max()
        assert err < 1e-12
    Tneg = toeplitz.galerkin_blocks(-ds, BRICK, K298)
    assert np.abs(Tneg - Tp.transpose(0, 2, 1)).max() / np.abs(Tp).max() < 1e-12


def test_sixty_unique_entries():
    """The N blocks have 60 distinct entries per offset (Sec. V, 60 unique
    tensors for PWL): on a generic offset exactly 60 distinct values up to
    sign remain."""
    T = toeplitz.galerkin_blocks(np.array([[3, 2, 1]]), BRICK, K298)[0]
    v = np.sort(T.reshape(-1))
    v = v[np.abs(v) > 1e-14 * np.abs(T).max()]
    v = v[np.argsort(v.real + 1e-3 * v.imag)]
    # cluster values that agree up to sign to 1e-9 relative (the basis swap
    # flips the sign of pulse/linear pairs)
    clusters = []
    for z in v:
        if not any(min(abs(z - c), abs(z + c)) <= 1e-9 * abs(c) for c in clusters):
            clusters.append(z)
    assert len(clusters) == 60


def test_far_blocks_match_unreduced_6d_quadrature():
    """Separated voxels: the reduced charge form equals the plain 6-D Gauss
    integral of N^l (k0^2 delta + grad grad) g N^l' (eq. 34a), all 144 entries."""
    for d in [(2, 0, 0), (2, 1, 0), (0, -2, 3), (3, 2, 1)]:
        A = toeplitz.galerkin_blocks(np.array([d]), BRICK, K298)[0]
        B = unreduced.block_6d(d, BRICK, K298, n=8)
        assert np.abs(A - B).max() / np.abs(B).max() < 1e-9, d


def test_quadrature_converged():
    ds = np.concatenate([NEAR[:8], MID])
    A = toeplitz.galerkin_blocks(ds, BRICK, K298)
    B = toeplitz.galerkin_blocks(ds, BRICK, K298, duffy_order=18, order_scale=1.4)
    assert np.abs(A - B).max() / np.abs(B).max() < 1e-12


def test_far_field_point_dipole_limit():
    """Far apart, the PWC block tends to dV^2 (k0^2 I + grad grad) g(d Delta);
    the relative difference is O((Delta/R)^2) + O((k0 Delta)^2), so use an
    electrically tiny voxel to see the geometric term shrink."""
    errs = []
    k = 1.0
    for n in (6, 12, 24):
        d = np.array([n, 0, 0])
        T = toeplitz.galerkin_blocks(d[None], CUBE, k)[0]
        pwc = T[0::4, 0::4]
        ref = np.prod(CUBE) ** 2 * unreduced.dyadic_green((d * np.array(CUBE))[None], k)[0]
        errs.append(np.abs(pwc - ref).max() / np.abs(ref).max())
    assert errs[0] < 1e-2 and errs[1] < errs[0] / 3 and errs[2] < errs[1] / 3


def test_gram_closed_form():
    """eq. 33: int N^l N^l over a voxel = dV (l=1), dV/12 (l=2..4); checked
    with quadrature."""
    x, w = np.polynomial.legendre.leggauss(3)
    D = np.array(BRICK)
    t = 0.5 * D[0] * x
    ref = np.prod(D) * np.sum(0.5 * w * (t / D[0]) ** 2)
    G = physics.gram_diag(*BRICK)
    assert G[0] == pytest.approx(np.prod(D), rel=1e-15)
    assert G[1] == pytest.approx(ref, rel=1e-14)
