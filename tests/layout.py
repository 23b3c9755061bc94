"""Layout conversions between the oracle ([a, ix, iy, iz]) and the library
((nrhs, 12, Nz, Ny, Nx), per-voxel (Nz, Ny, Nx)); no arithmetic of the method."""
import numpy as np

# representative (p, l, q, l') of unique entry u = 10 * pq + ll (p <= q, l <= l')
_P = [0, 0, 0, 1, 1, 2]
_Q = [0, 1, 2, 1, 2, 2]
_L = [1, 1, 1, 1, 2, 2, 2, 3, 3, 4]
_LP = [1, 2, 3, 4, 2, 3, 4, 3, 4, 4]
UNIQUE_AB = [(4 * _P[pq] + _L[ll] - 1, 4 * _Q[pq] + _LP[ll] - 1) for pq in range(6) for ll in range(10)]


def vec_to_lib(x):
    """[12, Nx, Ny, Nz] -> [12, Nz, Ny, Nx]"""
    return np.ascontiguousarray(np.asarray(x).transpose(0, 3, 2, 1))


def vec_from_lib(x):
    return np.ascontiguousarray(np.asarray(x).transpose(0, 3, 2, 1))


def vox_to_lib(v):
    return np.ascontiguousarray(np.asarray(v).transpose(2, 1, 0))


def unique_from_full(T):
    """Full oracle blocks [12, 12, 2Nx-1, 2Ny-1, 2Nz-1] -> unique [60, Nz, Ny, Nx], d >= 0."""
    _, _, sx, sy, sz = T.shape
    Nx, Ny, Nz = (sx + 1) // 2, (sy + 1) // 2, (sz + 1) // 2
    out = np.zeros((60, Nz, Ny, Nx), dtype=np.complex128)
    for u, (a, b) in enumerate(UNIQUE_AB):
        out[u] = T[a, b, Nx - 1:, Ny - 1:, Nz - 1:].transpose(2, 1, 0)
    return out


def unique_from_octant(Toct):
    """Oracle octant blocks [12, 12, Nx, Ny, Nz] -> unique [60, Nz, Ny, Nx]."""
    return np.stack([Toct[a, b].transpose(2, 1, 0) for (a, b) in UNIQUE_AB])


def relerr(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / np.abs(b).max())
