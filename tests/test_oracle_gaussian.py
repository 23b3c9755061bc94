"""The oracle's Galerkin blocks (Sec. III-B/C, eq. 25a, 33, 34a, 42) at the
touching and coincident offsets, pinned by a second numerical route that
shares nothing with the first: ``oracle.gaussian`` expands g in powers of R
and integrates 1/R through its Gaussian representation, with exact 1-D
factors (no boxes, no Duffy maps, no Gauss-Legendre rules).  The second route
is itself pinned by the closed-form static box potential, the cube's static
self term, the unreduced 6-D quadrature of the dyadic kernel on separated
voxels, and its own convergence in the one remaining quadrature (over t)."""
import itertools

import numpy as np
import pytest

from oracle import gaussian, physics, toeplitz, unreduced
from tests.test_oracle_toeplitz import _box_potential, _gauss_box

K298 = physics.k0(298e6)
BRICK = (0.005, 0.004, 0.003)
CUBE = (0.005, 0.005, 0.005)
NEAR27 = np.array(list(itertools.product((-1, 0, 1), repeat=3)))


def _blockwise_err(A, B):
    return max(float(np.abs(A[i] - B[i]).max() / np.abs(B[i]).max()) for i in range(len(B)))


@pytest.mark.parametrize("k0", [0.0, K298])
def test_near_blocks_two_routes_agree(k0):
    """All 27 offsets with max |d_i| <= 1 (coincident, face-, edge- and
    corner-touching voxels), all 144 entries of each block, brick voxel:
    the oracle's reduced Duffy quadrature equals the Gaussian route."""
    A = toeplitz.galerkin_blocks(NEAR27, BRICK, k0)
    B = gaussian.blocks(NEAR27, BRICK, k0)
    err = _blockwise_err(A, B)
    print("near blocks, k0 = %g: %.2e" % (k0, err))
    assert err < 1e-9


def test_near_scalar_and_charge_parts_agree():
    """The two pieces of the block separately (scalar S^{ll'} and charge
    C^{pl,ql'}), at 298 MHz."""
    for part in ("S", "C"):
        A = toeplitz.galerkin_blocks(NEAR27, BRICK, K298, part=part)
        B = gaussian.blocks(NEAR27, BRICK, K298, part=part)
        assert _blockwise_err(A, B) < 1e-9, part


def test_gaussian_route_t_quadrature_converged():
    ds = NEAR27[::3]
    A = gaussian.blocks(ds, BRICK, K298, step=0.05)
    B = gaussian.blocks(ds, BRICK, K298, step=0.1)
    assert _blockwise_err(A, B) < 1e-12


@pytest.mark.parametrize("Delta", [(1.0, 1.0, 1.0), (1.0, 0.8, 1.3)])
def test_gaussian_scalar_block_matches_closed_form(Delta):
    """S^{11}(d) at k0 = 0 against (1/4 pi) int_{V_m} of the closed-form box
    potential of V_n."""
    ds = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 0], [1, 1, 1], [2, 1, 0]])
    S = gaussian.blocks(ds, Delta, 0.0, part='S')
    D = np.array(Delta)
    for i, d in enumerate(ds):
        lo_m = d * D - D / 2
        X, W = _gauss_box(48, lo_m, lo_m + D)
        ref = np.sum(W * _box_potential(X, -D / 2, D / 2)) / (4 * np.pi)
        assert abs(S[i, 0, 0] - ref) / ref < 1e-9, (d, S[i, 0, 0], ref)


def test_gaussian_static_self_term_cube():
    """Cube at k0 = 0: N^{p1,p1}(0) = 2 dV / 3 (cubic symmetry and the trace
    identity give the charge part dV / 3)."""
    T = gaussian.blocks(np.array([[0, 0, 0]]), CUBE, 0.0)[0]
    dv = np.prod(CUBE)
    for p in range(3):
        assert abs(T[4 * p, 4 * p] - 2 * dv / 3) / dv < 1e-12


def test_gaussian_far_blocks_match_unreduced():
    """Separated voxels at 298 MHz: the Gaussian route (charge form, power
    series of g) equals the plain 6-D Gauss integral of N^l (k0^2 delta +
    grad grad) g N^l' with no integration by parts, all 144 entries."""
    for d in [(2, 0, 0), (2, 1, 0), (0, -2, 3)]:
        A = gaussian.blocks(np.array([d]), BRICK, K298)[0]
        B = unreduced.block_6d(d, BRICK, K298, n=8)
        assert np.abs(A - B).max() / np.abs(B).max() < 1e-9, d


def test_gaussian_route_at_higher_frequency():
    """k0 Delta about 0.3 (a 3 GHz field on 5 mm voxels): more terms of the
    power series of g, still equal to the oracle's blocks."""
    k0 = physics.k0(3e9)
    ds = NEAR27[::4]
    assert _blockwise_err(toeplitz.galerkin_blocks(ds, BRICK, k0), gaussian.blocks(ds, BRICK, k0)) < 1e-9
