"""The operator product without device allocation (vie_apply_noalloc)
against vie_apply on the same context: same kernels and launch shapes, so
the results agree bit for bit.  Two calls in a row, the second on a smaller
grid (the fixed workspace keeps the first call's contents), and a request
above the fixed workspace size is refused before any launch."""
import sys

import numpy as np
import pytest

import vie_inputs as vi
from tests.layout import vec_to_lib, vox_to_lib

pytestmark = pytest.mark.gpu

F = 298e6


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


def _setup(vie, N, D, seed, nc=12):
    c = vie.Context(0)
    if nc != 12:
        c.set_basis(nc)
    c.set_grid(N, D, F)
    e, s = vi.ellipsoid_phantom(N, D, seed)
    c.set_contrast(vox_to_lib(e), vox_to_lib(s))
    return c


def _vectors(torch, c, nrhs, seed, dtype):
    xs = np.stack([vec_to_lib(vi.complex_normal(seed + r, (c.nc,) + c.N)) for r in range(nrhs)])
    return torch.from_numpy(xs).to("cuda", dtype).contiguous()


def _check_same(vie, torch, c, nrhs, seed):
    for dtype in (torch.complex64, torch.complex128):
        x = _vectors(torch, c, nrhs, seed, dtype)
        for op in (vie.OP_PREC, vie.OP_A, vie.OP_N):
            _say("  grid %s nc %d nrhs %d %s op %d" % (c.N, c.nc, nrhs, dtype, op))
            y_ref = torch.full_like(x, float("nan"))
            y_na = torch.full_like(x, float("nan"))
            c.apply(x, y_ref, op=op)
            c.apply_noalloc(x, y_na, op=op)
            torch.cuda.synchronize()
            assert torch.isfinite(torch.view_as_real(y_na)).all()
            assert torch.equal(y_ref, y_na)


def test_noalloc_matches_apply_two_calls(vie, torch):
    big = _setup(vie, (24, 20, 16), (0.005, 0.004, 0.006), 61)
    _check_same(vie, torch, big, 2, 62)
    small = _setup(vie, (7, 5, 6), (0.005,) * 3, 63)   # second call, smaller
    _check_same(vie, torch, small, 1, 64)
    pwc = _setup(vie, (9, 6, 5), (0.005,) * 3, 65, nc=3)
    _check_same(vie, torch, pwc, 3, 66)


def test_noalloc_refuses_oversize(vie, torch):
    c = vie.Context(0)
    c.set_grid((40, 40, 40), (0.005,) * 3, F)   # complex128: 74 MB of intermediates
    c.set_contrast(np.ones((40, 40, 40)), np.zeros((40, 40, 40)))
    x = torch.zeros(c.vec_shape(1), dtype=torch.complex128, device="cuda")
    y = torch.empty_like(x)
    with pytest.raises(vie.VieError) as ei:
        c.apply_noalloc(x, y, op=vie.OP_N)
    assert ei.value.code == vie.VIE_EINVAL
    x64 = torch.zeros(c.vec_shape(1), dtype=torch.complex64, device="cuda")   # 37 MB: fits
    y64 = torch.empty_like(x64)
    c.apply_noalloc(x64, y64, op=vie.OP_N)
    torch.cuda.synchronize()
    assert not bool(y64.abs().max())
    with pytest.raises(vie.VieError) as ei:
        c.apply_noalloc(x64, x64, op=vie.OP_N)   # overlapping x and y
    assert ei.value.code == vie.VIE_EINVAL


def test_noalloc_takes_no_device_memory(vie, torch):
    """Free device memory is unchanged by no-allocation products on a fresh
    context, while the first vie_apply on it grows the context workspace by
    the product's intermediates (which shows the measurement can see it)."""
    N = (40, 40, 40)
    c = _setup(vie, N, (0.005,) * 3, 67)
    x = _vectors(torch, c, 1, 68, torch.complex64)
    y = torch.empty_like(x)
    c.apply_noalloc(x, y, op=vie.OP_PREC)   # first dispatches (runtime set-up of the kernels)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(3):
        c.apply_noalloc(x, y, op=vie.OP_PREC)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    c.apply(x, y, op=vie.OP_PREC)
    torch.cuda.synchronize()
    free2 = torch.cuda.mem_get_info()[0]
    _say("  free memory change: noalloc %d B, apply %d B" % (free0 - free1, free1 - free2))
    assert free0 - free1 <= 0
    # the workspace grows from the set-up's 80^3 complex128 circulant (8 MB)
    # to the product's 37 MB of complex64 intermediates
    assert free1 - free2 >= 16 << 20
