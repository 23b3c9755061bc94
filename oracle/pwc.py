"""Piecewise-constant (PWC) discretisation (TEST INFRASTRUCTURE, see package doc).

The paper compares its PWL solver against the current-based VIE with one
constant basis function per voxel and vector component (Sec. I; Sec. V: 3
unknowns per voxel, 6 unique Toeplitz tensors).  That constant is the first
of the four scalar functions of the PWL basis (l = 1 in eq. 30), so the PWC
Galerkin system is the PWL system restricted to the unknowns a = 4 p:
operator blocks N^{(p,1),(q,1)}(d) (eq. 24-25 with l = l' = 1), Gram dV
(eq. 33 for l = 1), tested incident field e_t^{p1} (eq. 30), and the
preconditioned system P^-1 A x = x - tau G^-1 N x of Sec. IV-B with G = dV I.

Layout: vectors [3, Nx, Ny, Nz] with unknown p (x, y, z); blocks
[3, 3, 2Nx-1, 2Ny-1, 2Nz-1] indexed by d_i + N_i - 1 as for PWL.
"""
import numpy as np
import scipy.fft

from . import physics

# PWL unknown a = 4 p + (l - 1) of each PWC unknown p (l = 1)
PWL_INDEX = (0, 4, 8)


def blocks_from_pwl(T):
    """PWC blocks: the (p,1),(q,1) entries of the PWL blocks."""
    idx = np.array(PWL_INDEX)
    return T[idx[:, None], idx[None, :]]


def restrict(v):
    """The l = 1 coefficients of a PWL vector [12, ...] -> [3, ...]."""
    return v[list(PWL_INDEX)]


def direct_N(T3, x):
    """(N x)_m = sum_n T3(m - n) x_n over all voxel pairs (eq. 24-25)."""
    _, Nx, Ny, Nz = x.shape
    y = np.zeros_like(x, dtype=np.complex128)
    for dx in range(-Nx + 1, Nx):
        mx, nx = slice(max(0, dx), Nx + min(0, dx)), slice(max(0, -dx), Nx + min(0, -dx))
        for dy in range(-Ny + 1, Ny):
            my, ny = slice(max(0, dy), Ny + min(0, dy)), slice(max(0, -dy), Ny + min(0, -dy))
            for dz in range(-Nz + 1, Nz):
                mz, nz = slice(max(0, dz), Nz + min(0, dz)), slice(max(0, -dz), Nz + min(0, -dz))
                blk = T3[:, :, dx + Nx - 1, dy + Ny - 1, dz + Nz - 1]
                y[:, mx, my, mz] += np.tensordot(blk, x[:, nx, ny, nz], axes=(1, 0))
    return y


def spectrum(T3, M, workers=-1):
    """Circulant embedding on the M grid (T3(d) at index d mod M_i) and its
    forward 3-D DFT (Sec. IV-A)."""
    Nx, Ny, Nz = [(s + 1) // 2 for s in T3.shape[2:]]
    C = np.zeros((3, 3) + tuple(M), dtype=np.complex128)
    ix = np.arange(-Nx + 1, Nx) % M[0]
    iy = np.arange(-Ny + 1, Ny) % M[1]
    iz = np.arange(-Nz + 1, Nz) % M[2]
    C[:, :, ix[:, None, None], iy[None, :, None], iz[None, None, :]] = T3
    return scipy.fft.fftn(C, axes=(2, 3, 4), workers=workers)


def fft_N(Chat, x, workers=-1):
    """N x through zero padding, FFT, per-frequency 3 x 3 product, inverse FFT
    and crop (Sec. IV-A)."""
    M = Chat.shape[2:]
    _, Nx, Ny, Nz = x.shape
    xp = np.zeros((3,) + tuple(M), dtype=np.complex128)
    xp[:, :Nx, :Ny, :Nz] = x
    xh = scipy.fft.fftn(xp, axes=(1, 2, 3), workers=workers)
    yh = np.einsum('ab...,b...->a...', Chat, xh)
    return scipy.fft.ifftn(yh, axes=(1, 2, 3), workers=workers)[:, :Nx, :Ny, :Nz]


def apply_prec(T3, x, tau, Delta, Nx_fn=direct_N):
    """P^-1 A x = x - tau (N x) / dV (Sec. IV-B, eq. 17, with G = dV I)."""
    dv = Delta[0] * Delta[1] * Delta[2]
    return x - tau[None] * Nx_fn(T3, x) / dv


def apply_A(T3, x, epsr, chi, Delta, Nx_fn=direct_N):
    """A x = M_eps dV x - M_chi N x (eq. 24a with G = dV I)."""
    dv = Delta[0] * Delta[1] * Delta[2]
    return epsr[None] * dv * x - chi[None] * Nx_fn(T3, x)


def rhs_prec(e_t3, tau, Delta, freq_hz):
    """P^-1 b = c_e tau e_t / dV (eq. 24b, 31 with G = dV I)."""
    dv = Delta[0] * Delta[1] * Delta[2]
    return physics.c_e(freq_hz) * tau[None] * e_t3 / dv


def dense_prec_matrix(T3, tau, Delta):
    """Dense P^-1 A = I - M_tau N / dV, row and column index p * N_V + voxel
    (voxel in C order over (x, y, z))."""
    _, _, sx, sy, sz = T3.shape
    Nx, Ny, Nz = (sx + 1) // 2, (sy + 1) // 2, (sz + 1) // 2
    NV = Nx * Ny * Nz
    m = np.stack(np.meshgrid(np.arange(Nx), np.arange(Ny), np.arange(Nz), indexing='ij'), -1).reshape(-1, 3)
    d = m[:, None, :] - m[None, :, :]
    blk = T3[:, :, d[..., 0] + Nx - 1, d[..., 1] + Ny - 1, d[..., 2] + Nz - 1]   # [3,3,NV,NV]
    Nmat = blk.transpose(0, 2, 1, 3).reshape(3 * NV, 3 * NV)
    dv = Delta[0] * Delta[1] * Delta[2]
    rowscale = np.tile(tau.reshape(-1), 3) / dv
    return np.eye(3 * NV, dtype=np.complex128) - rowscale[:, None] * Nmat


def solve_dense(T3, tau, Delta, rhs_prec_):
    """Exact solution of the PWC system by LU; [3, Nx, Ny, Nz] in and out."""
    x = np.linalg.solve(dense_prec_matrix(T3, tau, Delta), rhs_prec_.reshape(-1))
    return x.reshape(rhs_prec_.shape)


def total_field(T3, x, e_t3, Delta, freq_hz, Nx_fn=direct_N):
    """Total field everywhere in the box through one operator product
    (Sec. IV-C): dV e = e_t + (N x - dV x) / c_e."""
    dv = Delta[0] * Delta[1] * Delta[2]
    return (e_t3 + (Nx_fn(T3, x) - dv * x) / physics.c_e(freq_hz)) / dv


def absorbed_power(x3, chi, Delta, freq_hz):
    """P_abs = 1/2 Re{ x^* (c_e M_chi)^-1 dV x } (eq. 44 with G = dV I)."""
    dv = Delta[0] * Delta[1] * Delta[2]
    ce = physics.c_e(freq_hz)
    m = chi != 0
    q = np.zeros(chi.shape, dtype=np.complex128)
    q[m] = 1.0 / (ce * chi[m])
    return 0.5 * dv * float(np.real(np.sum(np.conj(x3) * x3 * q[None])))


def power_density(e3, sigma):
    """p_abs = 1/2 sigma |e|^2 of the constant field of each voxel (Sec. V-C)."""
    return 0.5 * sigma * np.sum(np.abs(e3) ** 2, axis=0)
