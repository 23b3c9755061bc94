"""Galerkin operator products (TEST INFRASTRUCTURE, see package doc).

Layout: vectors are [12, Nx, Ny, Nz] complex128 with unknown a = 4 p + (l-1)
(eq. 30 ordering); block tensors are [12, 12, 2Nx-1, 2Ny-1, 2Nz-1] indexed by
d_i + N_i - 1 (eq. 42).

* ``direct_N``: (N x)_m = sum_n T(m - n) x_n, the plain O(N_V^2) voxel-pair
  sum of eq. (24)-(25), regrouped by offset d = m - n.
* ``apply_prec``: left-preconditioned operator of Sec. IV-B,
  P^-1 A x = x - tau (G^-1 N x) with P = M_eps G, A = M_eps G - M_chi N
  (eq. 17, 24a).
* ``apply_A``: the unpreconditioned A x = eps_r G x - chi (N x) (eq. 24a).
* ``fft_N``: the same product through circulant embedding on an M grid and
  FFT (Sec. IV-A).  The embedding places T(d) at index d mod M_i on each axis
  (offsets that do not occur stay zero); that makes the circulant product equal
  the Toeplitz one on the original grid.
"""
import numpy as np
import scipy.fft

from . import physics


def direct_N(T, x):
    """(N x)_m = sum_n T(m - n) x_n over all voxel pairs (eq. 24-25, 42)."""
    _, Nx, Ny, Nz = x.shape
    y = np.zeros_like(x, dtype=np.complex128)

    def rng(d, n):
        # observation indices m and source indices m - d inside [0, n)
        return slice(max(0, d), n + min(0, d)), slice(max(0, -d), n + min(0, -d))

    for dx in range(-Nx + 1, Nx):
        mx, nx = rng(dx, Nx)
        for dy in range(-Ny + 1, Ny):
            my, ny = rng(dy, Ny)
            for dz in range(-Nz + 1, Nz):
                mz, nz = rng(dz, Nz)
                blk = T[:, :, dx + Nx - 1, dy + Ny - 1, dz + Nz - 1]
                y[:, mx, my, mz] += np.tensordot(blk, x[:, nx, ny, nz], axes=(1, 0))
    return y


def per_unknown(v):
    """Broadcast a per-voxel [Nx, Ny, Nz] array to the 12 unknowns."""
    return np.broadcast_to(v, (12,) + v.shape)


def apply_prec(T, x, tau, Delta, Nx_fn=direct_N):
    """P^-1 A x = x - tau G^-1 (N x)  (eq. 17 with P = M_eps G, Sec. IV-B)."""
    G = physics.gram_vector(*Delta)
    return x - per_unknown(tau) * (Nx_fn(T, x) / G[:, None, None, None])


def apply_A(T, x, epsr, chi, Delta, Nx_fn=direct_N):
    """A x = M_eps G x - M_chi N x (eq. 24a)."""
    G = physics.gram_vector(*Delta)
    return per_unknown(epsr) * G[:, None, None, None] * x - per_unknown(chi) * Nx_fn(T, x)


def rhs_prec(e_t, tau, Delta, freq_hz):
    """P^-1 b = c_e tau G^-1 e_t, with b = c_e chi e_t (eq. 24b, 31)."""
    G = physics.gram_vector(*Delta)
    return physics.c_e(freq_hz) * per_unknown(tau) * e_t / G[:, None, None, None]


def rhs(e_t, chi, freq_hz):
    """b = c_e chi e_t (eq. 31)."""
    return physics.c_e(freq_hz) * per_unknown(chi) * e_t


# ---------------------------------------------------------------------------
# circulant / FFT route (Sec. IV-A)
# ---------------------------------------------------------------------------
def circulant(T, M):
    """Embed the blocks T(d), d in (-N, N)^3, into circulant tensors on the M
    grid: C[:, :, j] = T(d) with j_i = d_i mod M_i (requires M_i >= 2N_i - 1)."""
    Nx, Ny, Nz = [(s + 1) // 2 for s in T.shape[2:]]
    assert all(M[i] >= 2 * n - 1 for i, n in enumerate((Nx, Ny, Nz)))
    C = np.zeros((12, 12) + tuple(M), dtype=np.complex128)
    ix = np.arange(-Nx + 1, Nx) % M[0]
    iy = np.arange(-Ny + 1, Ny) % M[1]
    iz = np.arange(-Nz + 1, Nz) % M[2]
    C[:, :, ix[:, None, None], iy[None, :, None], iz[None, None, :]] = T
    return C


def circulant_spectrum(T, M, workers=-1):
    """Forward 3-D DFT of the circulant tensors (unnormalised, e^{-2 pi i})."""
    return scipy.fft.fftn(circulant(T, M), axes=(2, 3, 4), workers=workers)


def fft_N(Chat, x, workers=-1):
    """(N x) by zero padding to the M grid, FFT, per-frequency 12 x 12 product,
    inverse FFT and crop (Sec. IV-A)."""
    M = Chat.shape[2:]
    _, Nx, Ny, Nz = x.shape
    xp = np.zeros((12,) + tuple(M), dtype=np.complex128)
    xp[:, :Nx, :Ny, :Nz] = x
    xh = scipy.fft.fftn(xp, axes=(1, 2, 3), workers=workers)
    yh = np.einsum('ab...,b...->a...', Chat, xh)
    y = scipy.fft.ifftn(yh, axes=(1, 2, 3), workers=workers)
    return y[:, :Nx, :Ny, :Nz]


# ---------------------------------------------------------------------------
# symmetries of the blocks (used to build the full offset range from the
# d >= 0 octant once the tests have checked them on directly computed blocks)
# ---------------------------------------------------------------------------
def reflection_signs(axis):
    """sigma_axis(a) for the 12 unknowns: reflecting the axis flips the vector
    component along it and the linear function along it (eq. 20, 22)."""
    s = np.ones(12)
    for p in range(3):
        for l in range(1, 5):
            a = 4 * p + l - 1
            if p == axis:
                s[a] *= -1
            if l == axis + 2:
                s[a] *= -1
    return s


def full_from_octant(Toct):
    """[12,12,Nx,Ny,Nz] blocks for d >= 0 -> [12,12,2Nx-1,2Ny-1,2Nz-1] using
    T(.., -d_i, ..) = sigma_i(a) sigma_i(b) T(.., d_i, ..)."""
    _, _, Nx, Ny, Nz = Toct.shape
    T = np.zeros((12, 12, 2 * Nx - 1, 2 * Ny - 1, 2 * Nz - 1), dtype=np.complex128)
    for sx in (1, -1):
        for sy in (1, -1):
            for sz in (1, -1):
                sgn = np.ones((12, 12))
                for axis, s in enumerate((sx, sy, sz)):
                    if s < 0:
                        r = reflection_signs(axis)
                        sgn = sgn * np.outer(r, r)
                ix = Nx - 1 + sx * np.arange(Nx)
                iy = Ny - 1 + sy * np.arange(Ny)
                iz = Nz - 1 + sz * np.arange(Nz)
                T[:, :, ix[:, None, None], iy[None, :, None], iz[None, None, :]] = sgn[:, :, None, None, None] * Toct
    return T
