"""Linear solves (TEST INFRASTRUCTURE, see package doc).

* ``dense_prec_matrix`` + ``solve_dense``: the exact discrete solution of the
  left-preconditioned system P^-1 A x = P^-1 b (eq. 17, 24) by LU, for tiny
  grids.
* ``gmres``: restarted GMRES(m) (Sec. V: inner 50, outer 200), modified
  Gram-Schmidt Arnoldi, Givens rotations, x0 = 0, stopping on the relative
  residual ||r|| / ||b|| of the system it is given.
"""
import numpy as np

from . import physics


def dense_prec_matrix(T, tau, Delta):
    """Dense P^-1 A = I - M_tau G^-1 N as a (12 N_V) x (12 N_V) matrix, row and
    column index a * N_V + voxel (voxel in C order over (x, y, z))."""
    _, _, sx, sy, sz = T.shape
    Nx, Ny, Nz = (sx + 1) // 2, (sy + 1) // 2, (sz + 1) // 2
    NV = Nx * Ny * Nz
    m = np.stack(np.meshgrid(np.arange(Nx), np.arange(Ny), np.arange(Nz), indexing='ij'), -1).reshape(-1, 3)
    d = m[:, None, :] - m[None, :, :]
    blocks = T[:, :, d[..., 0] + Nx - 1, d[..., 1] + Ny - 1, d[..., 2] + Nz - 1]   # [12,12,NV,NV]
    Nmat = blocks.transpose(0, 2, 1, 3).reshape(12 * NV, 12 * NV)
    G = physics.gram_vector(*Delta)
    rowscale = (np.repeat(1.0 / G, NV) * np.tile(tau.reshape(-1), 12))
    return np.eye(12 * NV, dtype=np.complex128) - rowscale[:, None] * Nmat


def solve_dense(T, tau, Delta, rhs_prec):
    """Exact solution of P^-1 A x = P^-1 b; rhs and result as [12, Nx, Ny, Nz]."""
    A = dense_prec_matrix(T, tau, Delta)
    x = np.linalg.solve(A, rhs_prec.reshape(-1))
    return x.reshape(rhs_prec.shape)


def gmres(apply, b, restart=50, tol=1e-6, max_outer=200, x0=None):
    """Restarted GMRES(restart) for apply(x) = b.  Returns (x, info) with
    info = dict(iters, converged, history) and history the relative residual
    estimate after every inner step."""
    shape = b.shape
    bv = b.reshape(-1).astype(np.complex128)
    bnorm = np.linalg.norm(bv)
    x = np.zeros_like(bv) if x0 is None else x0.reshape(-1).astype(np.complex128).copy()
    hist = []
    iters = 0
    if bnorm == 0.0:
        return x.reshape(shape), dict(iters=0, converged=True, history=[0.0])
    for _ in range(max_outer):
        r = bv - apply(x.reshape(shape)).reshape(-1)
        beta = np.linalg.norm(r)
        if beta / bnorm <= tol:
            return x.reshape(shape), dict(iters=iters, converged=True, history=hist)
        V = np.zeros((restart + 1, bv.size), dtype=np.complex128)
        H = np.zeros((restart + 1, restart), dtype=np.complex128)
        cs = np.zeros(restart, dtype=np.complex128)
        sn = np.zeros(restart, dtype=np.complex128)
        g = np.zeros(restart + 1, dtype=np.complex128)
        g[0] = beta
        V[0] = r / beta
        k_done = 0
        for j in range(restart):
            w = apply(V[j].reshape(shape)).reshape(-1)
            for i in range(j + 1):                      # modified Gram-Schmidt
                H[i, j] = np.vdot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] != 0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):                          # previous rotations
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -np.conj(sn[i]) * H[i, j] + np.conj(cs[i]) * H[i + 1, j]
                H[i, j] = t
            den = np.sqrt(abs(H[j, j]) ** 2 + abs(H[j + 1, j]) ** 2)
            # rotation [[c, s], [-conj(s), conj(c)]] zeroing H[j+1, j]
            cs[j] = np.conj(H[j, j]) / den
            sn[j] = np.conj(H[j + 1, j]) / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            iters += 1
            k_done = j + 1
            hist.append(abs(g[j + 1]) / bnorm)
            if hist[-1] <= tol:
                break
        y = np.linalg.solve(np.triu(H[:k_done, :k_done]), g[:k_done])
        x = x + V[:k_done].T @ y
    r = bv - apply(x.reshape(shape)).reshape(-1)
    ok = np.linalg.norm(r) / bnorm <= tol
    return x.reshape(shape), dict(iters=iters, converged=bool(ok), history=hist)
