"""GPU parity of the HIP library against the oracle, through the C ABI.

Tolerances: operator products agree with the oracle's direct voxel-pair sum
within 1e-11 (complex128) and 1e-5 (complex64) relative (max-norm over the
result).  Block tensors assembled on the device agree with the oracle's
independent quadrature within 1e-10 relative to the largest entry of each
offset.  Solves are compared with the oracle's exact (dense LU) solution.
"""
import functools
import sys

import numpy as np
import pytest

import vie_inputs as vi
from oracle import incident, matvec, physics, post, solve, toeplitz
from tests.layout import relerr, unique_from_full, unique_from_octant, vec_from_lib, vec_to_lib, vox_to_lib

pytestmark = pytest.mark.gpu

F = 298e6
K = physics.k0(F)


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def vie(torch):
    import paper_1902_02196_amd as v
    return v


@functools.lru_cache(None)
def _full_blocks(N, D):
    return toeplitz.toeplitz_full(N, D, K)


def _ctx(vie, torch, N, D, T_full=None):
    c = vie.Context(0)
    c.set_grid(N, D, F)
    if T_full is not None:
        c.set_toeplitz(unique_from_full(T_full))
    return c


def _to_dev(torch, x_oracle, dtype):
    return torch.from_numpy(vec_to_lib(x_oracle)[None]).to(device="cuda", dtype=dtype).contiguous()


def _from_dev(y):
    return vec_from_lib(y[0].cpu().numpy())


CASES = [((4, 4, 4), (0.005, 0.005, 0.005)), ((5, 3, 6), (0.006, 0.005, 0.004)), ((8, 8, 8), (0.005,) * 3),
         ((1, 2, 3), (0.004, 0.006, 0.005)), ((7, 4, 9), (0.005, 0.004, 0.006))]


@pytest.mark.parametrize("N,D", CASES)
def test_matvec_N_parity_same_blocks(vie, torch, N, D):
    """FFT product on the device vs the direct voxel-pair sum, both fed the
    oracle's block tensors (ragged sizes, non-smooth 2N padded to smooth M)."""
    _say("matvec N parity %s" % (N,))
    T = _full_blocks(N, D)
    c = _ctx(vie, torch, N, D, T)
    x = vi.complex_normal(11, (12,) + N)
    ref = matvec.direct_N(T, x)
    for dtype, tol in ((torch.complex128, 1e-11), (torch.complex64, 1e-5)):
        xd = _to_dev(torch, x, dtype)
        yd = torch.empty_like(xd)
        c.apply(xd, yd, op=vie.OP_N)
        torch.cuda.synchronize()
        err = relerr(_from_dev(yd), ref)
        _say("  %s err %.3e" % (dtype, err))
        assert err < tol


@pytest.mark.parametrize("N,D", CASES[:3])
def test_device_assembly_matches_oracle(vie, torch, N, D):
    """Block tensors assembled on the device (closed-form axis kernels, own
    quadrature) vs the oracle's (quadrature-evaluated correlations)."""
    _say("assembly parity %s" % (N,))
    c = _ctx(vie, torch, N, D)
    lib = c.get_toeplitz()
    ref = unique_from_octant(toeplitz.toeplitz_octant(N, D, K))
    for iz in range(N[2]):
        for iy in range(N[1]):
            for ix in range(N[0]):
                a, b = lib[:, iz, iy, ix], ref[:, iz, iy, ix]
                assert np.abs(a - b).max() <= 1e-10 * np.abs(b).max(), (ix, iy, iz)


def test_device_assembly_far_offsets(vie, torch):
    """Sampled offsets in every Gauss-order band of the device assembly (up to
    max |d_i| = 39) vs the oracle's blocks at the same offsets."""
    from tests.layout import UNIQUE_AB
    N, D = (40, 24, 20), (0.005, 0.004, 0.006)
    c = _ctx(vie, torch, N, D)
    lib = c.get_toeplitz()
    offs = [(2, 0, 0), (2, 2, 2), (0, 1, 2), (3, 1, 0), (4, 4, 4), (5, 0, 0), (8, 8, 8), (7, 2, 5), (9, 0, 0),
            (16, 3, 1), (12, 12, 12), (17, 0, 0), (25, 10, 3), (39, 23, 19), (0, 0, 19), (0, 23, 0), (33, 1, 18)]
    ref = toeplitz.galerkin_blocks(np.array(offs), D, K)
    for (ix, iy, iz), blk in zip(offs, ref):
        b = np.array([blk[a, bb] for a, bb in UNIQUE_AB])
        a = lib[:, iz, iy, ix]
        assert np.abs(a - b).max() <= 1e-10 * np.abs(b).max(), (ix, iy, iz)


@pytest.mark.parametrize("N,D", CASES[:2])
def test_preconditioned_and_plain_operators(vie, torch, N, D):
    """P^-1 A (eq. 17) and A (eq. 24a) with a heterogeneous phantom, library
    assembly, vs the oracle with its own blocks."""
    _say("operators %s" % (N,))
    c = _ctx(vie, torch, N, D)
    e, s = vi.ellipsoid_phantom(N, D, 3)
    c.set_contrast(vox_to_lib(e), vox_to_lib(s))
    T = _full_blocks(N, D)
    x = vi.complex_normal(12, (12,) + N)
    er, ch, ta = physics.eps_r(e, s, F), physics.chi(e, s, F), physics.tau(e, s, F)
    for op, ref in ((vie.OP_PREC, matvec.apply_prec(T, x, ta, D)), (vie.OP_A, matvec.apply_A(T, x, er, ch, D))):
        for dtype, tol in ((torch.complex128, 1e-10), (torch.complex64, 1e-5)):
            xd = _to_dev(torch, x, dtype)
            yd = torch.empty_like(xd)
            c.apply(xd, yd, op=op)
            torch.cuda.synchronize()
            err = relerr(_from_dev(yd), ref)
            _say("  op %d %s err %.3e" % (op, dtype, err))
            assert err < tol


def test_batched_apply_equals_single(vie, torch):
    """Several right-hand sides in one launch give the same result as one at
    a time (bitwise: no cross-RHS reductions in the product)."""
    N, D = (6, 5, 4), (0.005,) * 3
    c = _ctx(vie, torch, N, D)
    e, s = vi.ellipsoid_phantom(N, D, 4)
    c.set_contrast(vox_to_lib(e), vox_to_lib(s))
    xs = np.stack([vec_to_lib(vi.complex_normal(20 + r, (12,) + N)) for r in range(3)])
    for dtype in (torch.complex64, torch.complex128):
        xd = torch.from_numpy(xs).to("cuda", dtype)
        yd = torch.empty_like(xd)
        c.apply(xd, yd, op=vie.OP_PREC)
        for r in range(3):
            y1 = torch.empty_like(xd[r:r + 1])
            c.apply(xd[r:r + 1].contiguous(), y1, op=vie.OP_PREC)
            assert torch.equal(y1[0], yd[r])


def test_planewave_and_rhs(vie, torch):
    N, D = (5, 4, 6), (0.006, 0.005, 0.004)
    c = _ctx(vie, torch, N, D)
    e, s = vi.sphere(N, D, 0.012, 50.0, 0.7)
    c.set_contrast(vox_to_lib(e), vox_to_lib(s))
    et = torch.empty(c.vec_shape(1), dtype=torch.complex128, device="cuda")
    c.incident_planewave(et)
    ref = incident.planewave_tested(N, D, K)
    assert relerr(_from_dev(et), ref) < 1e-13
    rhs = torch.empty_like(et)
    c.rhs_prec(et, rhs)
    assert relerr(_from_dev(rhs), matvec.rhs_prec(ref, physics.tau(e, s, F), D, F)) < 1e-13


def test_dipole_rhs(vie, torch):
    N, D = (6, 5, 4), (0.005,) * 3
    c = _ctx(vie, torch, N, D)
    e, s = vi.ellipsoid_phantom(N, D, 5)
    c.set_contrast(vox_to_lib(e), vox_to_lib(s))
    pos, mom = vi.dipoles_on_cylinder(7, 2, 0.03, N[2] * D[2])
    et = torch.empty(c.vec_shape(2), dtype=torch.complex128, device="cuda")
    c.incident_dipoles(et, pos, mom, nq=6)
    chi = physics.chi(e, s, F)
    ref = incident.dipoles_tested(N, D, F, pos, mom, chi != 0, nq=6)
    for r in range(2):
        assert relerr(vec_from_lib(et[r].cpu().numpy()), ref[r]) < 1e-12


@pytest.mark.parametrize("mode,tol,bound,reorth", [(0, 1e-12, 1e-9, 0), (1, 1e-10, 1e-7, 0), (0, 1e-12, 1e-9, 1),
                                                   (1, 1e-10, 1e-7, 1)])
def test_solve_matches_dense(vie, torch, mode, tol, bound, reorth):
    """GMRES on the device (FP64, and FP32 + FP64 refinement; one or two
    Gram-Schmidt passes) vs the oracle's exact discrete solution by dense LU
    (4 x 4 x 4 sphere, config-1 material)."""
    _say("solve mode %d reorth %d" % (mode, reorth))
    N, D = (4, 4, 4), (0.005,) * 3
    T = _full_blocks(N, D)
    c = _ctx(vie, torch, N, D)
    e, s = vi.sphere(N, D, 0.0101, 50.0, 0.7)
    c.set_contrast(vox_to_lib(e), vox_to_lib(s))
    tau, chi = physics.tau(e, s, F), physics.chi(e, s, F)
    et = incident.planewave_tested(N, D, K)
    xref = solve.solve_dense(T, tau, D, matvec.rhs_prec(et, tau, D, F))
    etd = _to_dev(torch, et, torch.complex128)
    xd = torch.empty_like(etd)
    code, st = c.solve(etd, xd, mode=mode, tol=tol, restart=20, reorth=reorth)
    _say("  stats %s" % st[0])
    assert code == vie.VIE_OK and st[0]["converged"]
    err = relerr(_from_dev(xd), xref)
    _say("  err %.3e" % err)
    assert err < bound
    P = c.absorbed_power(xd)[0]
    assert abs(P - post.absorbed_power(xref, chi, D, F)) / abs(P) < 10 * bound


def test_total_field_matches_oracle(vie, torch):
    """Total field in the whole box (tissue and air) through one product
    (Sec. IV-C) vs the oracle's, on the same blocks; and at the exact
    discrete solution it equals x / (c_e chi) on the tissue voxels."""
    N, D = (5, 4, 6), (0.005, 0.006, 0.004)
    T = _full_blocks(N, D)
    c = _ctx(vie, torch, N, D, T)
    e, s = vi.ellipsoid_phantom(N, D, 33)
    c.set_contrast(vox_to_lib(e), vox_to_lib(s))
    x = vi.complex_normal(34, (12,) + N)
    et = incident.planewave_tested(N, D, K)
    xd, etd = _to_dev(torch, x, torch.complex128), _to_dev(torch, et, torch.complex128)
    out = torch.empty_like(xd)
    c.total_field(etd, xd, out)
    assert relerr(_from_dev(out), post.total_field(T, x, et, D, F)) < 1e-12
    # identity at the solution (4^3 sphere with air corners, dense LU)
    N, D = (4, 4, 4), (0.005,) * 3
    T = _full_blocks(N, D)
    c = _ctx(vie, torch, N, D, T)
    e, s = vi.sphere(N, D, 0.0101, 50.0, 0.7)
    c.set_contrast(vox_to_lib(e), vox_to_lib(s))
    tau, chi = physics.tau(e, s, F), physics.chi(e, s, F)
    et = incident.planewave_tested(N, D, K)
    xref = solve.solve_dense(T, tau, D, matvec.rhs_prec(et, tau, D, F))
    xd, etd = _to_dev(torch, xref, torch.complex128), _to_dev(torch, et, torch.complex128)
    tot, fld = torch.empty_like(xd), torch.empty_like(xd)
    c.total_field(etd, xd, tot)
    c.fields(xd, fld)
    m = chi != 0
    assert 0 < m.sum() < m.size
    a, b = _from_dev(tot)[:, m], _from_dev(fld)[:, m]
    assert np.abs(a - b).max() < 1e-9 * np.abs(b).max()


def test_fields_and_power_density(vie, torch):
    N, D = (4, 3, 5), (0.005,) * 3
    c = _ctx(vie, torch, N, D)
    e, s = vi.ellipsoid_phantom(N, D, 9)
    c.set_contrast(vox_to_lib(e), vox_to_lib(s))
    x = vi.complex_normal(13, (12,) + N)
    xd = _to_dev(torch, x, torch.complex128)
    ed = torch.empty_like(xd)
    c.fields(xd, ed)
    chi = physics.chi(e, s, F)
    eref = post.fields_from_currents(x, chi, F)
    assert relerr(_from_dev(ed), eref) < 1e-14
    pd = torch.empty((1,) + tuple(reversed(N)), dtype=torch.float64, device="cuda")
    c.power_density(ed, pd)
    assert relerr(pd[0].cpu().numpy().transpose(2, 1, 0), post.power_density(eref, s)) < 1e-13
    P = c.absorbed_power(xd)[0]
    assert abs(P - post.absorbed_power(x, chi, D, F)) / abs(P) < 1e-12


def test_errors_are_reported(vie, torch):
    c = vie.Context(0)
    with pytest.raises(vie.VieError):
        c.set_grid((4, 4, 4), (0.005, -1.0, 0.005), F)
    c.set_grid((4, 4, 4), (0.005,) * 3, F)
    e = np.ones((4, 4, 4))
    s = np.zeros((4, 4, 4))
    s[0, 0, 0] = np.nan
    with pytest.raises(vie.VieError) as ei:
        c.set_contrast(e, s)
    assert ei.value.code == vie.VIE_ENAN
    x = torch.zeros(c.vec_shape(1), dtype=torch.complex128, device="cuda")
    with pytest.raises(vie.VieError) as ei:
        c.apply(x, torch.empty_like(x), op=vie.OP_PREC)   # no contrast yet
    assert ei.value.code == vie.VIE_ESTATE


def test_autotuned_shapes_keep_results(vie, torch):
    """Every launch shape the autotuner may pick computes the same product
    (to rounding: the x-pass variants sum the block terms in another order)."""
    N, D = (16, 12, 10), (0.005,) * 3
    c = _ctx(vie, torch, N, D)
    e, s = vi.ellipsoid_phantom(N, D, 8)
    c.set_contrast(vox_to_lib(e), vox_to_lib(s))
    x = torch.from_numpy(np.stack([vec_to_lib(vi.complex_normal(30 + r, (12,) + N)) for r in range(2)]))
    for dtype, tol in ((torch.complex64, 2e-6), (torch.complex128, 1e-13)):
        xd = x.to("cuda", dtype)
        y0 = torch.empty_like(xd)
        c.apply(xd, y0, op=vie.OP_PREC)
        choice, ms = c.autotune(vie.C64 if dtype == torch.complex64 else vie.C128, 2)
        _say("  autotune %s: %s %.3f ms" % (dtype, choice, ms))
        y1 = torch.empty_like(xd)
        c.apply(xd, y1, op=vie.OP_PREC)
        assert float((y1 - y0).abs().max() / y0.abs().max()) < tol


@pytest.mark.parametrize("N", [(16, 12, 10), (24, 20, 12), (5, 3, 6)])
def test_every_launch_shape_matches_oracle(vie, torch, N):
    """Each x-pass variant and strided-pass tile, installed explicitly, gives
    the oracle's FFT product (complex64; complex128 where the variant exists)."""
    D = (0.005, 0.004, 0.006)
    c = _ctx(vie, torch, N, D)
    T = toeplitz.toeplitz_full(N, D, K)
    c.set_toeplitz(unique_from_full(T))
    xs = [vi.complex_normal(40 + r, (12,) + N) for r in range(3)]
    Ch = matvec.circulant_spectrum(T, tuple(2 * n for n in N))
    ref = [matvec.fft_N(Ch, x) for x in xs]
    x = torch.from_numpy(np.stack([vec_to_lib(v) for v in xs]))
    shapes = [dict(variant=v, sib_blocks=sb, tile_z=tz, tile_y=ty)
              for v, sb in ((0, 1), (0, 2), (0, 4), (1, 1), (2, 1), (3, 1), (4, 1), (5, 1))
              for tz in (8, 16, 32) for ty in (8, 16, 32)]
    ran = 0
    for dtype, prec, tol in ((torch.complex64, vie.C64, 1e-5), (torch.complex128, vie.C128, 1e-11)):
        xd = x.to("cuda", dtype)
        for sh in shapes:
            try:
                c.set_tuning(sh, prec, 3)
            except vie.VieError:
                continue   # shape not available for this grid or precision
            y = torch.empty_like(xd)
            c.apply(xd, y, op=vie.OP_N)
            for r in range(3):
                err = relerr(_from_dev(y[r:r + 1]), ref[r])
                assert err < tol, (dtype, sh, r, err)
            ran += 1
    _say("  %d shapes checked" % ran)
    assert ran >= 8


@pytest.mark.parametrize("N", [(4, 4, 384), (4, 256, 4)])
def test_long_strided_tiles_match_oracle(vie, torch, N):
    """Strided passes of length 768 (z) and 512 (y), where tiles of 4 and 8
    pencils (32 and 64 bytes in complex64, less than a cache line) are
    compiled beside 16 and 32: every tile, installed explicitly, gives the
    oracle's FFT product in both precisions."""
    D = (0.005, 0.004, 0.006)
    _say("long strided tiles %s" % (N,))
    c = _ctx(vie, torch, N, D)
    Toct = toeplitz.toeplitz_octant(N, D, K)
    c.set_toeplitz(unique_from_octant(Toct))
    T = matvec.full_from_octant(Toct)
    xs = [vi.complex_normal(60 + r, (12,) + N) for r in range(2)]
    Ch = matvec.circulant_spectrum(T, tuple(2 * n for n in N))
    ref = [matvec.fft_N(Ch, x) for x in xs]
    x = torch.from_numpy(np.stack([vec_to_lib(v) for v in xs]))
    ran = 0
    for dtype, prec, tol in ((torch.complex64, vie.C64, 1e-5), (torch.complex128, vie.C128, 1e-11)):
        xd = x.to("cuda", dtype)
        for tz in (4, 8, 16, 32):
            for ty in (4, 8, 16, 32):
                try:
                    c.set_tuning(dict(variant=1, sib_blocks=1, tile_z=tz, tile_y=ty), prec, 2)
                except vie.VieError:
                    continue   # tile not available for this length or precision
                y = torch.empty_like(xd)
                c.apply(xd, y, op=vie.OP_N)
                for r in range(2):
                    err = relerr(_from_dev(y[r:r + 1]), ref[r])
                    assert err < tol, (dtype, tz, ty, r, err)
                ran += 1
    _say("  %d tile pairs checked" % ran)
    assert ran >= 16


def test_shared_grid_matches_own_assembly(vie, torch):
    """A context sharing another's operator (vie_share_grid) computes the same
    products bitwise as one that assembled its own, keeps working after the
    source context is gone, and refuses to overwrite the shared blocks."""
    N, D = (6, 5, 7), (0.005, 0.004, 0.006)
    a = _ctx(vie, torch, N, D)
    b = vie.Context(0)
    b.share_grid(a)
    assert b.fft_size == a.fft_size
    own = _ctx(vie, torch, N, D)
    e, s = vi.ellipsoid_phantom(N, D, 21)
    for c in (b, own):
        c.set_contrast(vox_to_lib(e), vox_to_lib(s))
    x = torch.from_numpy(vec_to_lib(vi.complex_normal(22, (12,) + N))[None]).cuda()
    yb, yo = torch.empty_like(x), torch.empty_like(x)
    with pytest.raises(vie.VieError):
        b.set_toeplitz(np.zeros((60, N[2], N[1], N[0]), dtype=np.complex128))
    a.close()
    b.apply(x, yb, op=vie.OP_PREC)
    own.apply(x, yo, op=vie.OP_PREC)
    assert torch.equal(yb, yo)



def test_degenerate_cases(vie, torch):
    """Edge cases of the method: a single voxel (fft length 2, generic
    kernels) against the oracle's direct sum, and solved against dense LU with
    a Krylov space used up within one cycle; no contrast, where P^-1 A is the
    identity and a zero right-hand side solves to zero at once; zero right-hand
    side counts are refused."""
    N, D = (1, 1, 1), (0.004, 0.005, 0.006)
    T = _full_blocks(N, D)
    c = _ctx(vie, torch, N, D, T)
    assert c.fft_size == (2, 2, 2)
    x = vi.complex_normal(51, (12,) + N)
    ref = matvec.direct_N(T, x)
    for dtype, tol in ((torch.complex128, 1e-12), (torch.complex64, 1e-6)):
        xd = _to_dev(torch, x, dtype)
        yd = torch.empty_like(xd)
        c.apply(xd, yd, op=vie.OP_N)
        assert relerr(_from_dev(yd), ref) < tol

    N, D = (6, 5, 4), (0.005,) * 3
    c = _ctx(vie, torch, N, D)
    c.set_contrast(np.ones((N[2], N[1], N[0])), np.zeros((N[2], N[1], N[0])))   # air: chi = 0
    x = torch.from_numpy(vec_to_lib(vi.complex_normal(52, (12,) + N))[None]).cuda()
    y = torch.empty_like(x)
    c.apply(x, y, op=vie.OP_PREC)
    assert torch.equal(x, y)
    et = torch.zeros_like(x)
    xs = torch.full_like(x, 1.0)
    code, st = c.solve(et, xs, mode=vie.SOLVE_FP32_IR)
    assert code == vie.VIE_OK and st[0]["iterations"] == 0
    assert not bool(xs.abs().max())
    # one voxel with contrast: the 12 unknowns use the Krylov space up within
    # one restart cycle, so the last vectors vanish up to rounding
    N1, D1 = (1, 1, 1), (0.004, 0.005, 0.006)
    T1 = _full_blocks(N1, D1)
    c1 = _ctx(vie, torch, N1, D1, T1)
    e1, s1 = np.full(N1, 50.0), np.full(N1, 0.7)
    c1.set_contrast(vox_to_lib(e1), vox_to_lib(s1))
    tau1 = physics.tau(e1, s1, F)
    et1 = incident.planewave_tested(N1, D1, K)
    xref = solve.solve_dense(T1, tau1, D1, matvec.rhs_prec(et1, tau1, D1, F))
    for mode, tol, bound in ((vie.SOLVE_FP64, 1e-13, 1e-10), (vie.SOLVE_FP32_IR, 1e-11, 1e-8)):
        etd = _to_dev(torch, et1, torch.complex128)
        xd = torch.empty_like(etd)
        code, st = c1.solve(etd, xd, mode=mode, tol=tol, restart=20)
        _say("  one voxel, mode %d: %s" % (mode, st[0]))
        assert code == vie.VIE_OK and st[0]["converged"]
        assert relerr(_from_dev(xd), xref) < bound
    with pytest.raises(vie.VieError) as ei:
        c.apply(x[:0], y[:0], op=vie.OP_PREC)
    assert ei.value.code == vie.VIE_EINVAL
