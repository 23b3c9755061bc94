"""Brute-force 6-D Gauss quadrature of the dyadic kernel (TEST INFRASTRUCTURE).

For voxels that neither overlap nor touch, the Galerkin block of eq. (34a) is
an ordinary smooth 6-D integral:

    T^{pl,ql'}(d) = int_{V_m} int_{V_n} N^l(r) [(k0^2 delta_pq + d_p d_q) g](r - r') N^{l'}(r') dr' dr

with g(R) = exp(-i k0 R) / (4 pi R) (eq. 10) differentiated analytically:

    d_p d_q g = g [(-k0^2 + 3 i k0 / R + 3 / R^2) Rp Rq - (i k0 / R + 1 / R^2) delta_pq],

Rp, Rq the components of the unit vector R_hat.  No dimension reduction, no
integration by parts: this is the independent check of the charge-form
reduction in ``oracle.toeplitz`` for well-separated voxels.
"""
import numpy as np


def dyadic_green(Rvec, k0):
    """(k0^2 I + grad grad) g at separation vectors Rvec [..., 3] -> [..., 3, 3]."""
    R = np.linalg.norm(Rvec, axis=-1)
    Rh = Rvec / R[..., None]
    g = np.exp(-1j * k0 * R) / (4.0 * np.pi * R)
    a = -k0 * k0 + 3j * k0 / R + 3.0 / R ** 2
    b = 1j * k0 / R + 1.0 / R ** 2
    I = np.eye(3)
    gg = g[..., None, None] * (a[..., None, None] * Rh[..., :, None] * Rh[..., None, :] - b[..., None, None] * I)
    return gg + (k0 * k0) * g[..., None, None] * I


def block_6d(d, Delta, k0, n=6):
    """T(d) [12, 12] by n^6-point tensor Gauss-Legendre over the two voxels."""
    x, w = np.polynomial.legendre.leggauss(n)
    Delta = np.asarray(Delta, dtype=np.float64)
    pts = [0.5 * Delta[i] * x for i in range(3)]            # local coords
    wts = [0.5 * Delta[i] * w for i in range(3)]
    U = np.stack(np.meshgrid(*pts, indexing='ij'), -1).reshape(-1, 3)
    WU = np.einsum('i,j,k->ijk', *wts).reshape(-1)
    # scalar basis values N^l at the local points (eq. 20)
    Nl = np.stack([np.ones(U.shape[0]), U[:, 0] / Delta[0], U[:, 1] / Delta[1], U[:, 2] / Delta[2]], 1)
    off = np.asarray(d, dtype=np.float64) * Delta
    out = np.zeros((12, 12), dtype=np.complex128)
    # chunk over test points to bound memory
    for s in range(0, U.shape[0], 512):
        Rv = off + U[s:s + 512, None, :] - U[None, :, :]
        K = dyadic_green(Rv, k0)                             # [nu, nv, 3, 3]
        wl = (WU[s:s + 512, None] * Nl[s:s + 512])           # [nu, 4]
        wr = (WU[:, None] * Nl)                              # [nv, 4]
        blk = np.einsum('ul,uvpq,vm->plqm', wl, K, wr)
        out += blk.reshape(12, 12)
    return out


def curl_green(Rvec, k0):
    """The curl kernel: (curl (g q_hat))_p = sum_k eps_pkq d_k g, returned as
    [..., 3, 3] with entry [p, q] = sum_k eps_pkq d_k g(R),
    d_k g = -(1 + i k0 R) exp(-i k0 R) / (4 pi R^2) R_k / R."""
    R = np.linalg.norm(Rvec, axis=-1)
    dg = -(1.0 + 1j * k0 * R) * np.exp(-1j * k0 * R) / (4.0 * np.pi * R ** 2)
    G = dg[..., None] * Rvec / R[..., None]               # grad g
    out = np.zeros(Rvec.shape[:-1] + (3, 3), dtype=np.complex128)
    for p, k, q, s in ((0, 1, 2, 1), (1, 2, 0, 1), (2, 0, 1, 1), (0, 2, 1, -1), (2, 1, 0, -1), (1, 0, 2, -1)):
        out[..., p, q] += s * G[..., k]
    return out


def curl_block_6d(d, Delta, k0, n=6):
    """K(d) [12, 12] = < f^{pl}, curl S f^{ql'} > by n^6-point tensor
    Gauss-Legendre over two separated voxels (no integration by parts)."""
    x, w = np.polynomial.legendre.leggauss(n)
    Delta = np.asarray(Delta, dtype=np.float64)
    pts = [0.5 * Delta[i] * x for i in range(3)]
    wts = [0.5 * Delta[i] * w for i in range(3)]
    U = np.stack(np.meshgrid(*pts, indexing='ij'), -1).reshape(-1, 3)
    WU = np.einsum('i,j,k->ijk', *wts).reshape(-1)
    Nl = np.stack([np.ones(U.shape[0]), U[:, 0] / Delta[0], U[:, 1] / Delta[1], U[:, 2] / Delta[2]], 1)
    off = np.asarray(d, dtype=np.float64) * Delta
    out = np.zeros((12, 12), dtype=np.complex128)
    for s in range(0, U.shape[0], 512):
        Rv = off + U[s:s + 512, None, :] - U[None, :, :]
        K = curl_green(Rv, k0)
        wl = (WU[s:s + 512, None] * Nl[s:s + 512])
        wr = (WU[:, None] * Nl)
        out += np.einsum('ul,uvpq,vm->plqm', wl, K, wr).reshape(12, 12)
    return out
