"""Tucker (low multilinear rank) compression of the Toeplitz-defining
tensors (TEST INFRASTRUCTURE, see the package docstring).

Sec. III-C ends by noting that the tensors N^{pl,ql'}(m) of eq. 43, m in
[0, N)^3, keep a low multilinear rank, so that they can be stored as a
Tucker decomposition, a small core times one factor matrix per axis (and
Sec. V leaves their memory out of the footprint for that reason).  The paper
does not fix the algorithm; this module follows the reading the library
uses:

* sequentially truncated HOSVD in the mode order x, y, z: for each mode the
  left singular vectors of the mode unfolding of the tensor as compressed so
  far, the smallest singular values dropped while the sum of their squares
  stays within tol^2 ||T||_F^2 / 3, and the tensor projected onto the kept
  vectors before the next mode;
* then T ~ core x_x U_x x_y U_y x_z U_z with orthonormal factors, and the
  error is exactly the square root of the sum of the dropped squares (the
  three projections are orthogonal), at most tol ||T||_F.

Arrays are indexed [x, y, z] like the oracle's blocks; plain numpy SVD of
the unfoldings (the library works from Gram matrices instead).
"""
import numpy as np


def unfold(X, mode):
    """Mode-`mode` unfolding: the axis `mode` first, the others flattened."""
    return np.moveaxis(X, mode, 0).reshape(X.shape[mode], -1)


def mode_product(X, M, mode):
    """X x_mode M: sum_n M[r, n] X[..., n, ...] along axis `mode`."""
    return np.moveaxis(np.tensordot(M, X, axes=(1, mode)), 0, mode)


def truncation_rank(s, budget):
    """Fewest leading singular values s (descending) whose dropped tail has
    sum of squares <= budget; at least 1."""
    sq = np.asarray(s, dtype=np.float64) ** 2
    tail = np.concatenate([np.cumsum(sq[::-1])[::-1], [0.0]])   # tail[k] = sum_{j >= k} s_j^2
    r = int(np.argmax(tail <= budget))
    return max(r, 1)


def st_hosvd(X, tol):
    """Sequentially truncated HOSVD of a 3-D tensor at relative Frobenius
    tolerance tol.  Returns (core, [U_x, U_y, U_z], dropped) where dropped[i]
    is the sum of the squared singular values dropped at mode i."""
    X = np.asarray(X, dtype=np.complex128)
    budget = tol ** 2 * float(np.vdot(X, X).real) / 3.0
    core = X
    factors, dropped = [], []
    for mode in range(3):
        U, s, _ = np.linalg.svd(unfold(core, mode), full_matrices=False)
        r = truncation_rank(s, budget)
        factors.append(U[:, :r])
        dropped.append(float(np.sum(s[r:] ** 2)))
        core = mode_product(core, U[:, :r].conj().T, mode)
    return core, factors, dropped


def reconstruct(core, factors):
    """core x_x U_x x_y U_y x_z U_z."""
    X = core
    for mode, U in enumerate(factors):
        X = mode_product(X, U, mode)
    return X


def compressed_size(core, factors):
    """Complex values stored: the core and the three factor matrices."""
    return core.size + sum(U.size for U in factors)
