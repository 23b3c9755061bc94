"""Current-based VIE with polarisation and magnetisation currents, the J-M
formulation for objects with magnetic contrast (TEST INFRASTRUCTURE, see
the package docstring).

Sec. II: with j = c_e chi_e e and m = c_m chi_m h (eq. 6-7, c_e = i w eps0,
c_m = i w mu0) the scattered fields are (eq. 13)

    e_sca = (1/c_e)(N - I) j - K m,      h_sca = K j + (1/c_m)(N - I) m,

and the currents solve A [j; m] = C M_chi [e_inc; h_inc] (eq. 14) with

    A = [[M_eps - M_chi_e N,  c_e M_chi_e K],
         [-c_m M_chi_m K,     M_mu - M_chi_m N]]                (eq. 15).

Discretised on the PWL basis as the dielectric equation (contrasts constant
per voxel, applied to the tested products): x = [x_j; x_m], 24 coefficients
per voxel (the electric 12 first, each ordered a = 4 p + (l - 1)),

    (A x)_j = eps_r G x_j - chi_e (N x_j) + c_e chi_e (K x_m)
    (A x)_m = -c_m chi_m (K x_j) + mu_r G x_m - chi_m (N x_m)
    b       = [c_e chi_e e_t; c_m chi_m h_t]

and, left-preconditioned like Sec. IV-B with P = diag(M_eps G, M_mu G),

    P^-1 A x = [x_j - tau_e G^-1 (N x_j - c_e K x_m);
                x_m - tau_m G^-1 (N x_m + c_m K x_j)],   tau = chi / (1 + chi).

Vectors [24, Nx, Ny, Nz]; N blocks from ``toeplitz`` (part 'N'), K blocks
from part 'K', both [12, 12, 2Nx-1, 2Ny-1, 2Nz-1].
"""
import numpy as np

from . import physics
from .matvec import direct_N


def _split(x):
    return x[:12], x[12:]


def apply_A(TN, TK, x, epsr, chie, mur, chim, Delta, freq_hz, Nx_fn=direct_N, Kx_fn=direct_N):
    """(A x) of the discrete eq. 14-15."""
    G = physics.gram_vector(*Delta)[:, None, None, None]
    ce, cm = physics.c_e(freq_hz), physics.c_m(freq_hz)
    xj, xm = _split(x)
    yj = epsr * G * xj - chie * Nx_fn(TN, xj) + ce * chie * Kx_fn(TK, xm)
    ym = -cm * chim * Kx_fn(TK, xj) + mur * G * xm - chim * Nx_fn(TN, xm)
    return np.concatenate([yj, ym])


def apply_prec(TN, TK, x, taue, taum, Delta, freq_hz, Nx_fn=direct_N, Kx_fn=direct_N):
    """P^-1 A x with P = diag(M_eps G, M_mu G)."""
    G = physics.gram_vector(*Delta)[:, None, None, None]
    ce, cm = physics.c_e(freq_hz), physics.c_m(freq_hz)
    xj, xm = _split(x)
    yj = xj - taue * (Nx_fn(TN, xj) - ce * Kx_fn(TK, xm)) / G
    ym = xm - taum * (Nx_fn(TN, xm) + cm * Kx_fn(TK, xj)) / G
    return np.concatenate([yj, ym])


def rhs(e_t, h_t, chie, chim, freq_hz):
    """b = C M_chi [e_t; h_t] (eq. 14, tested)."""
    return np.concatenate([physics.c_e(freq_hz) * chie * e_t, physics.c_m(freq_hz) * chim * h_t])


def rhs_prec(e_t, h_t, taue, taum, Delta, freq_hz):
    """P^-1 b = [c_e tau_e G^-1 e_t; c_m tau_m G^-1 h_t]."""
    G = physics.gram_vector(*Delta)[:, None, None, None]
    return np.concatenate([physics.c_e(freq_hz) * taue * e_t / G, physics.c_m(freq_hz) * taum * h_t / G])


def _dense_blocks(T):
    """Dense (12 N_V) x (12 N_V) matrix of a block tensor, index a * N_V + voxel."""
    _, _, sx, sy, sz = T.shape
    Nx, Ny, Nz = (sx + 1) // 2, (sy + 1) // 2, (sz + 1) // 2
    NV = Nx * Ny * Nz
    m = np.stack(np.meshgrid(np.arange(Nx), np.arange(Ny), np.arange(Nz), indexing='ij'), -1).reshape(-1, 3)
    d = m[:, None, :] - m[None, :, :]
    blocks = T[:, :, d[..., 0] + Nx - 1, d[..., 1] + Ny - 1, d[..., 2] + Nz - 1]
    return blocks.transpose(0, 2, 1, 3).reshape(12 * NV, 12 * NV)


def dense_prec_matrix(TN, TK, taue, taum, Delta, freq_hz):
    """Dense P^-1 A, (24 N_V) x (24 N_V), row and column index
    (12 h + a) * N_V + voxel with h = 0 for j, 1 for m."""
    Nm, Km = _dense_blocks(TN), _dense_blocks(TK)
    n = Nm.shape[0]
    NV = n // 12
    G = physics.gram_vector(*Delta)
    ce, cm = physics.c_e(freq_hz), physics.c_m(freq_hz)
    se = np.repeat(1.0 / G, NV) * np.tile(taue.reshape(-1), 12)
    sm = np.repeat(1.0 / G, NV) * np.tile(taum.reshape(-1), 12)
    A = np.eye(2 * n, dtype=np.complex128)
    A[:n, :n] -= se[:, None] * Nm
    A[:n, n:] += ce * se[:, None] * Km
    A[n:, :n] -= cm * sm[:, None] * Km
    A[n:, n:] -= sm[:, None] * Nm
    return A


def solve_dense(TN, TK, taue, taum, Delta, freq_hz, b_prec):
    A = dense_prec_matrix(TN, TK, taue, taum, Delta, freq_hz)
    return np.linalg.solve(A, b_prec.reshape(-1)).reshape(b_prec.shape)


def fields(x, chie, chim, freq_hz):
    """e = x_j / (c_e chi_e) where chi_e != 0, h = x_m / (c_m chi_m) where
    chi_m != 0 (eq. 6), zero elsewhere; [24, ...] (e first)."""
    xj, xm = _split(x)
    out = np.zeros_like(x)
    ce, cm = physics.c_e(freq_hz), physics.c_m(freq_hz)
    me, mm = chie != 0, chim != 0
    out[:12][:, me] = xj[:, me] / (ce * chie[me])
    out[12:][:, mm] = xm[:, mm] / (cm * chim[mm])
    return out


def absorbed_power(x, chie, chim, Delta, freq_hz):
    """P_abs = 1/2 Re{x_j^* (c_e M_chi_e)^-1 G x_j} + 1/2 Re{x_m^* (c_m M_chi_m)^-1 G x_m},
    i.e. 1/2 w eps0 int eps'' |e|^2 + 1/2 w mu0 int mu'' |h|^2 (eq. 44 and its
    magnetic counterpart)."""
    G = physics.gram_vector(*Delta)[:, None, None, None]
    xj, xm = _split(x)
    P = 0.0
    for xx, chi, c in ((xj, chie, physics.c_e(freq_hz)), (xm, chim, physics.c_m(freq_hz))):
        m = chi != 0
        q = np.zeros(chi.shape, dtype=np.complex128)
        q[m] = 1.0 / (c * chi[m])
        P += 0.5 * float(np.real(np.sum(np.conj(xx) * G * xx * q[None])))
    return P
