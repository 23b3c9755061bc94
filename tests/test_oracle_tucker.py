"""Pins of the oracle's Tucker compression (Sec. III-C, last paragraph: the
Toeplitz-defining tensors of eq. 43 have low multilinear rank): the helpers
against their index definitions, exact recovery of a tensor built with a
known multilinear rank, full-rank reconstruction, the error of the
sequentially truncated HOSVD equal to the dropped singular values and within
the tolerance on the physical tensors, orthonormal factors, ranks that grow
as the tolerance shrinks, and compression of the Green-function tensors."""
import numpy as np
import pytest

import vie_inputs as vi
from oracle import physics, toeplitz, tucker

K298 = physics.k0(298e6)


def _rand(shape, seed):
    return vi.complex_normal(seed, shape)


def test_unfold_and_mode_product_by_definition():
    X = _rand((3, 4, 5), 1)
    M = _rand((2, 4), 2)
    Y = tucker.mode_product(X, M, 1)
    ref = np.zeros((3, 2, 5), dtype=np.complex128)
    for i in range(3):
        for r in range(2):
            for k in range(5):
                ref[i, r, k] = sum(M[r, n] * X[i, n, k] for n in range(4))
    assert np.abs(Y - ref).max() < 1e-13
    U = tucker.unfold(X, 2)
    assert U.shape == (5, 12)
    for k in range(5):
        assert np.array_equal(U[k], X[:, :, k].reshape(-1))


def test_truncation_rank_counts_the_dropped_tail():
    s = np.array([4.0, 2.0, 1.0, 0.5])
    assert tucker.truncation_rank(s, 0.0) == 4
    assert tucker.truncation_rank(s, 0.25) == 3     # drop 0.5^2
    assert tucker.truncation_rank(s, 1.25) == 2     # drop 1 + 0.25
    assert tucker.truncation_rank(s, 1.2) == 3
    assert tucker.truncation_rank(s, 100.0) == 1    # at least one kept


def test_known_multilinear_rank_recovered():
    """core (2, 3, 4) times random tall factors: the HOSVD finds ranks
    (2, 3, 4) and reconstructs the tensor."""
    G = _rand((2, 3, 4), 3)
    A, B, C = _rand((9, 2), 4), _rand((7, 3), 5), _rand((8, 4), 6)
    X = tucker.reconstruct(G, [A, B, C])
    core, U, dropped = tucker.st_hosvd(X, 1e-12)
    assert core.shape == (2, 3, 4)
    assert np.abs(tucker.reconstruct(core, U) - X).max() < 1e-12 * np.abs(X).max()


def test_full_rank_is_exact_and_factors_orthonormal():
    X = _rand((5, 6, 7), 7)
    core, U, dropped = tucker.st_hosvd(X, 0.0)
    assert core.shape == (5, 6, 7)
    assert np.abs(tucker.reconstruct(core, U) - X).max() < 1e-12
    for M in U:
        assert np.abs(M.conj().T @ M - np.eye(M.shape[1])).max() < 1e-13


@pytest.mark.parametrize("tol", [1e-2, 1e-4, 1e-6])
def test_error_equals_dropped_and_meets_tolerance(tol):
    """On Galerkin blocks of a 12^3 grid (pulse-pulse xx and a
    linear-linear xy entry): ||T - T_hat|| equals the square root of the
    dropped squares (the projections are orthogonal) and is within tol ||T||."""
    N, D = (12, 12, 12), (0.005, 0.004, 0.006)
    T = toeplitz.toeplitz_octant(N, D, K298)
    for a, b in ((0, 0), (1, 5), (2, 10)):
        X = T[a, b]
        core, U, dropped = tucker.st_hosvd(X, tol)
        err = np.linalg.norm(tucker.reconstruct(core, U) - X)
        nx = np.linalg.norm(X)
        assert abs(err ** 2 - sum(dropped)) <= 1e-9 * nx ** 2
        assert err <= tol * nx * (1 + 1e-12)


def test_ranks_grow_as_tolerance_shrinks_and_compress():
    """The Green-function tensors compress: at 1e-6 every rank of the 16^3
    pulse-pulse tensor stays below the grid extent, and ranks never shrink
    as the tolerance does."""
    N, D = (16, 16, 16), (0.005,) * 3
    X = toeplitz.toeplitz_octant(N, D, K298)[0, 0]
    prev = (0, 0, 0)
    for tol in (1e-2, 1e-3, 1e-4, 1e-5, 1e-6):
        core, U, _ = tucker.st_hosvd(X, tol)
        r = core.shape
        assert all(a >= b for a, b in zip(r, prev))
        prev = r
    assert all(v < 16 for v in prev)
    assert tucker.compressed_size(core, U) < X.size / 2
