"""Serving (continuous batching) on the GPU through the C ABI.

Requests of different grids, materials, frequencies, precisions and dipole
counts are solved once each alone (one slot) and once all together (several
slots, overlapping on the device).  Every kernel of the path is free of
atomics on the result, so a request's solution and absorbed power are
bitwise the same alone and in the mix.  The smallest request is also checked
against the oracle's dense solution for the same dipole excitation, and a
PWC request against the oracle's dense PWC solution.
"""
import sys

import numpy as np
import pytest

import vie_inputs as vi
from oracle import incident, matvec, physics, post, pwc, solve, toeplitz
from tests.layout import relerr, vec_from_lib, vox_to_lib

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def vie():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1902_02196_amd as v
    return v


def _requests():
    out = []
    # (N, Delta, freq, (eps, sigma) [x, y, z], dipole seed, n dipoles, mode, tol)
    N, D = (4, 4, 4), (0.005,) * 3
    out.append((N, D, 298e6, vi.sphere(N, D, 0.0101, 50.0, 0.7), 11, 1, 0, 1e-12))
    N = (6, 5, 4)
    out.append((N, D, 128e6, vi.ellipsoid_phantom(N, D, 5), 12, 2, 1, 1e-8))
    N = (8, 8, 8)
    out.append((N, (0.004,) * 3, 298e6, vi.sphere(N, (0.004,) * 3, 0.015, 40.0, 0.5), 13, 3, 1, 1e-6))
    N = (5, 7, 6)
    out.append((N, (0.006, 0.005, 0.004), 298e6, vi.ellipsoid_phantom(N, (0.006, 0.005, 0.004), 6), 14, 1, 0,
                1e-9))
    N, D = (4, 4, 4), (0.005,) * 3
    out.append((N, D, 298e6, vi.sphere(N, D, 0.0101, 50.0, 0.7), 11, 1, 1, 1e-10))
    return out


def _submit(srv, req):
    N, D, f, (e, s), seed, n, mode, tol = req
    pos, mom = vi.dipoles_on_cylinder(seed, n, 0.04, N[2] * D[2])
    return srv.submit(N, D, f, vox_to_lib(e), vox_to_lib(s), pos, mom, mode=mode, tol=tol, restart=30,
                      want_x=True)


def _check_done(info):
    assert info["done"] == 1
    assert info["status"] == 0, info["message"]
    assert info["t_arrival"] <= info["t_start"] <= info["t_end"]


def test_same_result_alone_and_in_mix(vie):
    reqs = _requests()
    alone = []
    srv = vie.Server(0, hbm_budget=8 << 30, max_slots=1)
    cached = []
    for q in reqs:
        rid = _submit(srv, q)
        srv.wait()
        info, p, x = srv.result(rid)
        _check_done(info)
        _say("alone %d: iters %d res %.2e p %s cached %d" % (rid, info["iterations"], info["rel_residual"], p,
                                                           info["operator_cached"]))
        alone.append((p.copy(), x.copy()))
        cached.append(info["operator_cached"])
    # the last request repeats the first one's grid: its operator is reused
    assert cached == [0, 0, 0, 0, 1]
    st = srv.stats()
    assert st["operator_hits"] == 1 and st["operator_misses"] == 4 and st["operator_cache_bytes"] > 0
    srv.close()

    srv = vie.Server(0, hbm_budget=8 << 30, max_slots=4)
    ids = [_submit(srv, q) for q in reqs]
    srv.wait()
    st = srv.stats()
    _say("mix stats %s" % st)
    assert st["completed"] == len(reqs) and st["queued"] == 0 and st["running"] == 0
    assert 2 <= st["peak_running"] <= 4
    for rid, (p0, x0) in zip(ids, alone):
        info, p, x = srv.result(rid)
        _check_done(info)
        assert np.array_equal(p, p0)
        assert np.array_equal(x, x0)
    srv.close()


def test_served_solution_matches_oracle(vie):
    N, D, f, (e, s), seed, n, mode, tol = _requests()[0]
    srv = vie.Server(0, hbm_budget=1 << 30, max_slots=2)
    rid = _submit(srv, _requests()[0])
    srv.wait()
    info, p, x = srv.result(rid)
    _check_done(info)
    srv.close()
    K = physics.k0(f)
    T = toeplitz.toeplitz_full(N, D, K)
    tau, chi = physics.tau(e, s, f), physics.chi(e, s, f)
    pos, mom = vi.dipoles_on_cylinder(seed, n, 0.04, N[2] * D[2])
    et = incident.dipoles_tested(N, D, f, pos, mom, chi != 0, nq=4)[0]
    xref = solve.solve_dense(T, tau, D, matvec.rhs_prec(et, tau, D, f))
    err = relerr(vec_from_lib(x[0]), xref)
    _say("served vs dense: %.3e" % err)
    assert err < 1e-9
    pref = post.absorbed_power(xref, chi, D, f)
    assert abs(p[0] - pref) / abs(pref) < 1e-8


def test_pwc_request_matches_oracle(vie):
    """A PWC request (basis 3) served after a PWL request on the same grid
    takes the cached operator (the PWL operator serves both bases) and
    matches the oracle's dense PWC solution and absorbed power; the PWL
    request beside it matches its own dense solution; a basis other than
    12 or 3 is refused."""
    N, D, f = (4, 4, 4), (0.005,) * 3, 298e6
    e, s = vi.sphere(N, D, 0.0101, 50.0, 0.7)
    pos, mom = vi.dipoles_on_cylinder(11, 1, 0.04, N[2] * D[2])
    srv = vie.Server(0, hbm_budget=1 << 30, max_slots=2)
    r12 = srv.submit(N, D, f, vox_to_lib(e), vox_to_lib(s), pos, mom, mode=0, tol=1e-12, restart=30, want_x=True)
    srv.wait()
    r3 = srv.submit(N, D, f, vox_to_lib(e), vox_to_lib(s), pos, mom, mode=0, tol=1e-12, restart=30, want_x=True,
                    basis=3)
    srv.wait()
    info12, p12, x12 = srv.result(r12)
    info3, p3, x3 = srv.result(r3)
    _check_done(info12)
    _check_done(info3)
    assert x12.shape[1] == 12 and x3.shape[1] == 3
    assert info3["operator_cached"] == 1
    with pytest.raises(vie.VieError):
        srv.submit(N, D, f, vox_to_lib(e), vox_to_lib(s), pos, mom, basis=5)
    srv.close()
    K = physics.k0(f)
    T = toeplitz.toeplitz_full(N, D, K)
    tau, chi = physics.tau(e, s, f), physics.chi(e, s, f)
    et = incident.dipoles_tested(N, D, f, pos, mom, chi != 0, nq=4)[0]
    x12ref = solve.solve_dense(T, tau, D, matvec.rhs_prec(et, tau, D, f))
    T3 = pwc.blocks_from_pwl(T)
    x3ref = pwc.solve_dense(T3, tau, D, pwc.rhs_prec(pwc.restrict(et), tau, D, f))
    e12, e3 = relerr(vec_from_lib(x12[0]), x12ref), relerr(vec_from_lib(x3[0]), x3ref)
    p3ref = pwc.absorbed_power(x3ref, chi, D, f)
    _say("served PWL vs dense %.3e, PWC vs dense %.3e, PWC power %.4e (oracle %.4e)" % (e12, e3, p3[0], p3ref))
    assert e12 < 1e-9 and e3 < 1e-9
    assert abs(p3[0] - p3ref) / abs(p3ref) < 1e-8


def test_operator_cache_off_gives_same_result(vie):
    """With the operator cache disabled every request assembles its own
    operator, and the solution is bitwise the one obtained through the cache."""
    reqs = _requests()
    out = {}
    for cache in (True, False):
        srv = vie.Server(0, hbm_budget=4 << 30, max_slots=2)
        if not cache:
            srv.set_operator_cache(0)
        ids = [_submit(srv, reqs[0]), _submit(srv, reqs[0])]
        srv.wait()
        res = [srv.result(i) for i in ids]
        for info, _, _ in res:
            _check_done(info)
        st = srv.stats()
        _say("cache %s: hits %d misses %d" % (cache, st["operator_hits"], st["operator_misses"]))
        if not cache:
            assert st["operator_hits"] == 0 and st["operator_cache_bytes"] == 0
        out[cache] = [r[2].copy() for r in res]
        srv.close()
    for a, b in zip(out[True], out[False]):
        assert np.array_equal(a, b)


def test_operator_cache_eviction(vie):
    """With room for one operator only, alternating grids evict each other
    (no hits); with room for both, the repeats hit."""
    reqs = _requests()
    a, b = reqs[0], reqs[3]   # (4,4,4) and (5,7,6) grids
    for cap, want_hits in ((900 << 10, 0), (256 << 20, 2)):   # operators of 242016 and 746832 bytes
        srv = vie.Server(0, hbm_budget=8 << 30, max_slots=1)
        srv.set_operator_cache(cap)
        for q in (a, b, a, b):
            rid = _submit(srv, q)
            srv.wait()
            _check_done(srv.poll(rid))
        st = srv.stats()
        _say("cache %d B: hits %d misses %d bytes %d" % (cap, st["operator_hits"], st["operator_misses"],
                                                       st["operator_cache_bytes"]))
        assert st["operator_hits"] == want_hits
        assert st["operator_cache_bytes"] <= cap
        srv.close()


def test_admission_limits_and_errors(vie):
    N, D = (6, 6, 6), (0.005,) * 3
    e, s = vi.sphere(N, D, 0.012, 50.0, 0.7)
    pos, mom = vi.dipoles_on_cylinder(3, 1, 0.04, 0.03)
    fp = vie.footprint_bytes(*N, 1, vie.SOLVE_FP32_IR, 30)
    # budget for one request at a time: the second waits for the first
    srv = vie.Server(0, hbm_budget=int(1.5 * fp) + 4 * 12 * 216 * 16, max_slots=4)
    a = srv.submit(N, D, 298e6, vox_to_lib(e), vox_to_lib(s), pos, mom, restart=30)
    b = srv.submit(N, D, 298e6, vox_to_lib(e), vox_to_lib(s), pos, mom, restart=30)
    srv.wait()
    ia, ib = srv.poll(a), srv.poll(b)
    _check_done(ia)
    _check_done(ib)
    assert ib["t_start"] >= ia["t_end"]
    assert srv.stats()["peak_running"] == 1
    # larger than the whole budget: refused at submission
    big = (64, 64, 64)
    with pytest.raises(vie.VieError):
        srv.submit(big, D, 298e6, np.ones(big[::-1]), np.zeros(big[::-1]), pos, mom)
    # invalid material: the request finishes with an error status and message
    bad = vox_to_lib(e).copy()
    bad[0, 0, 0] = -1.0
    c = srv.submit(N, D, 298e6, bad, vox_to_lib(s), pos, mom)
    srv.wait()
    ic = srv.poll(c)
    assert ic["done"] == 1 and ic["status"] == vie.VIE_EINVAL and ic["message"]
    srv.close()
