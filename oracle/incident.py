"""Tested incident fields (TEST INFRASTRUCTURE, see package doc).

e_t^{pl}(m) = int_{V_m} N_m^l(r) e_inc^p(r) dV   (eq. 27, 30).

Grid convention (the paper does not fix the origin): the box is centred at the
origin, voxel centres at (n_i - (N_i - 1)/2) Delta_i, n_i = 0..N_i-1.
"""
import numpy as np

from . import physics


def voxel_centres(N, Delta):
    """Centre coordinates per axis (list of three 1-D arrays)."""
    return [(np.arange(N[i]) - 0.5 * (N[i] - 1)) * Delta[i] for i in range(3)]


def planewave_tested(N, Delta, k0, E0=1.0):
    """x-polarised plane wave E0 exp(-i k0 z) x_hat (Sec. V-A), tested in
    closed form: with a = dz/2 and z_m the voxel centre,
      e^{x,1} = dV exp(-i k0 z_m) sin(k0 a)/(k0 a)
      e^{x,4} = -2 i dx dy exp(-i k0 z_m) (sin(k0 a) - k0 a cos(k0 a)) / (k0^2 dz)
    and all other components zero (the x- and y-linear functions integrate a
    field constant in x, y to zero)."""
    dx, dy, dz = Delta
    cx, cy, cz = voxel_centres(N, Delta)
    a = 0.5 * dz
    ph = np.exp(-1j * k0 * cz)
    e = np.zeros((12,) + tuple(N), dtype=np.complex128)
    ka = k0 * a
    if ka == 0.0:
        l1 = dx * dy * dz * np.ones_like(ph)
        l4 = np.zeros_like(ph)
    else:
        l1 = dx * dy * dz * ph * np.sin(ka) / ka
        l4 = -2j * dx * dy * ph * (np.sin(ka) - ka * np.cos(ka)) / (k0 * k0 * dz)
    e[0] = E0 * l1[None, None, :]
    e[3] = E0 * l4[None, None, :]
    return e


def tested_by_quadrature(field_fn, N, Delta, nq=4, mask=None):
    """Generic tested field: Gauss-Legendre nq^3 points per voxel of
    N^l e^p (eq. 30).  field_fn(points [..., 3]) -> [..., 3] complex.
    Voxels where mask is False are left at zero."""
    x, w = np.polynomial.legendre.leggauss(nq)
    cx, cy, cz = voxel_centres(N, Delta)
    e = np.zeros((12,) + tuple(N), dtype=np.complex128)
    loc = [0.5 * Delta[i] * x for i in range(3)]
    wts = [0.5 * Delta[i] * w for i in range(3)]
    U = np.stack(np.meshgrid(*loc, indexing='ij'), -1).reshape(-1, 3)
    WU = np.einsum('i,j,k->ijk', *wts).reshape(-1)
    Nl = np.stack([np.ones(U.shape[0]), U[:, 0] / Delta[0], U[:, 1] / Delta[1], U[:, 2] / Delta[2]], 1)
    if mask is None:
        mask = np.ones(tuple(N), dtype=bool)
    idx = np.argwhere(mask)
    for s in range(0, idx.shape[0], 4096):
        ii = idx[s:s + 4096]
        centres = np.stack([cx[ii[:, 0]], cy[ii[:, 1]], cz[ii[:, 2]]], 1)
        P = centres[:, None, :] + U[None, :, :]
        E = field_fn(P)                                   # [nv, nq^3, 3]
        vals = np.einsum('vqp,q,ql->vpl', E, WU, Nl)       # [nv, 3, 4]
        e[:, ii[:, 0], ii[:, 1], ii[:, 2]] = vals.reshape(-1, 12).T
    return e


def planewave_field(P, k0, E0=1.0):
    E = np.zeros(P.shape[:-1] + (3,), dtype=np.complex128)
    E[..., 0] = E0 * np.exp(-1j * k0 * P[..., 2])
    return E


def dipole_field(P, r0, moment, freq_hz):
    """E of a Hertzian dipole with current moment I l (A m, vector) at r0, from
    e = (1/c_e)(k0^2 S + grad div S) j with j = I l delta(r - r0) (eq. 13 with
    N - I = k0^2 S + grad div S), time factor exp(+i w t):

      E = (1/c_e) exp(-i k R)/(4 pi R^3) [(k^2 R^2 - i k R - 1) m
                                         + (3 + 3 i k R - k^2 R^2)(R_hat . m) R_hat]
    """
    k = physics.k0(freq_hz)
    Rv = P - np.asarray(r0, dtype=np.float64)
    R = np.linalg.norm(Rv, axis=-1)
    Rh = Rv / R[..., None]
    m = np.asarray(moment, dtype=np.complex128)
    pre = np.exp(-1j * k * R) / (4.0 * np.pi * R ** 3) / physics.c_e(freq_hz)
    a = (k * k * R * R - 1j * k * R - 1.0)
    b = (3.0 + 3j * k * R - k * k * R * R) * (Rh @ m)
    return pre[..., None] * (a[..., None] * m + b[..., None] * Rh)


def dipoles_tested(N, Delta, freq_hz, positions, moments, mask, nq=4):
    """Tested fields [R, 12, Nx, Ny, Nz] for R dipoles, on voxels in mask."""
    out = []
    for r0, m in zip(positions, moments):
        out.append(tested_by_quadrature(lambda P: dipole_field(P, r0, m, freq_hz), N, Delta, nq, mask))
    return np.stack(out)
