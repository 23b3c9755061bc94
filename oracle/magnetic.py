"""Magnetic field, b1+ and magnetic energy from the solution (TEST
INFRASTRUCTURE, see the package docstring).

Paper Sec. II: h_tot = h_inc + K j (eq. 'tot_fields' b) with the curl
operator K u = curl S u (eq. 8b); Sec. III: K discretised on the PWL basis
like N, K^{pl,ql'}_{m,n} = < f_m^{pl}, K f_n^{ql'} > (eq. 25b), so the
tested total field satisfies  G h = h_t + K x  (x the current coefficients,
j = c_e chi e, h_t the tested incident magnetic field, eq. 30 with h in
place of e).  Sec. V-D: b1+ = mu0 (h_x + i h_y), W_m = 1/4 int mu |h|^2 dV,
w_m = 1/4 mu |h|^2 and the errors error_h1..3.

Layout as in ``matvec``: vectors [12, Nx, Ny, Nz], blocks
[12, 12, 2Nx-1, 2Ny-1, 2Nz-1]; the K blocks come from
``toeplitz.toeplitz_full(..., part='K')``.
"""
import numpy as np

from . import incident, physics
from .matvec import direct_N


def planewave_h_field(P, k0, E0=1.0):
    """H of the plane wave x_hat E0 exp(-i k0 z): y_hat E0 / eta0 exp(-i k0 z)
    (curl E = -i w mu0 H, time factor exp(+i w t))."""
    H = np.zeros(P.shape[:-1] + (3,), dtype=np.complex128)
    H[..., 1] = E0 / physics.ETA0 * np.exp(-1j * k0 * P[..., 2])
    return H


def dipole_h_field(P, r0, moment, freq_hz):
    """H of a Hertzian dipole (current moment I l, vector, at r0):
    h = K j = curl (g I l) = grad g x I l,
      H = (1 + i k R) exp(-i k R) / (4 pi R^2) (m x R_hat)."""
    k = physics.k0(freq_hz)
    Rv = P - np.asarray(r0, dtype=np.float64)
    R = np.linalg.norm(Rv, axis=-1)
    Rh = Rv / R[..., None]
    m = np.asarray(moment, dtype=np.complex128)
    pre = (1.0 + 1j * k * R) * np.exp(-1j * k * R) / (4.0 * np.pi * R ** 2)
    return pre[..., None] * np.cross(np.broadcast_to(m, Rh.shape), Rh)


def planewave_h_tested(N, Delta, k0, E0=1.0, nq=6):
    """Tested incident magnetic field of the x-polarised plane wave."""
    return incident.tested_by_quadrature(lambda P: planewave_h_field(P, k0, E0), N, Delta, nq)


def dipoles_h_tested(N, Delta, freq_hz, positions, moments, nq=4):
    """Tested incident magnetic fields [R, 12, Nx, Ny, Nz] of R dipoles, on
    every voxel (the sources lie outside the box)."""
    return np.stack([incident.tested_by_quadrature(lambda P, r0=r0, m=m: dipole_h_field(P, r0, m, freq_hz),
                                                   N, Delta, nq) for r0, m in zip(positions, moments)])


def total_h(TK, x, h_t, Delta, Kx_fn=direct_N):
    """Coefficients of h_tot = h_inc + K j on the PWL basis: G^-1 (h_t + K x)."""
    G = physics.gram_vector(*Delta)[:, None, None, None]
    return (h_t + Kx_fn(TK, x)) / G


def b1plus(h):
    """b1+ = mu0 (h_x + i h_y) (Sec. V-D), per scalar basis l: [4, Nx, Ny, Nz]."""
    return physics.MU0 * (h[0:4] + 1j * h[4:8])


def magnetic_energy_density(h, mu=physics.MU0):
    """Voxel average of w_m = 1/4 mu |h|^2 (Sec. V-D): with the Gram weights of
    eq. 33, 1/4 mu (sum_p |h^{p1}|^2 + 1/12 sum_{p, l>1} |h^{pl}|^2)."""
    w = np.tile(np.array([1.0, 1.0 / 12, 1.0 / 12, 1.0 / 12]), 3)[:, None, None, None]
    return 0.25 * mu * np.sum(w * np.abs(h) ** 2, axis=0)


def magnetic_energy(h, mask, Delta, mu=physics.MU0):
    """W_m = 1/4 int_V mu |h|^2 dV over the voxels in mask (Sec. V-D)."""
    return float(np.sum(magnetic_energy_density(h, mu)[mask]) * np.prod(Delta))


def rel_errors_h(W, W_ref, w, w_ref, h, h_ref, Delta):
    """error_h1, error_h2, error_h3 of Sec. V-D (error_h3 in the
    Gram-weighted norm, the L2 norm of the field over the voxels given)."""
    G = physics.gram_vector(*Delta)[:, None, None, None]
    e1 = abs(W - W_ref) / abs(W_ref)
    e2 = np.sum(np.abs(w - w_ref)) / np.sum(np.abs(w_ref))
    e3 = np.sqrt(np.sum(G * np.abs(h - h_ref) ** 2) / np.sum(G * np.abs(h_ref) ** 2))
    return e1, e2, e3
