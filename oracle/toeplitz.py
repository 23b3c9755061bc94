"""Galerkin blocks of the N operator for the discontinuous PWL voxel basis.

TEST INFRASTRUCTURE ONLY (see the package docstring).

What is computed (paper Sec. III-B/C, eq. 25a, 26, 32-34, 42-43): for a voxel
offset d = m - n (observation minus source voxel, in voxel units), the 12 x 12
block

    T^{pl,ql'}(d) = < f_m^{pl}, N f_n^{ql'} >,   N u = curl curl S u,

with f^{ql} = N^l q_hat, N^1 the voxel pulse and N^{2,3,4} = (x-x_n)/dx,
(y-y_n)/dy, (z-z_n)/dz times the pulse (eq. 19-22), S the convolution with
g(r) = exp(-i k0 |r|) / (4 pi |r|) (eq. 9-10).  Unknown index a = 4 p + (l-1).

Reading of the operator (the paper states eq. 8a, 10 and 13 but does not write
the split out): curl curl = grad div - Laplacian and (Laplacian + k0^2) g =
-delta give  N u = k0^2 S u + grad div S u + u,  hence

    T(d) = delta_{d,0} Gram + k0^2 delta_pq S^{ll'}(d) - C^{pl,ql'}(d)

with the Gram diagonal of eq. 33, the scalar block
S^{ll'}(d) = int int N^l(u) g(d*Delta + u - v) N^{l'}(v) du dv, and the
"charge" block C^{pl,ql'}(d) = int int (D_p N^l)(u) g(.) (D_q N^{l'})(v), where
D_p is the distributional derivative along axis p of the basis restricted to
its voxel (interior derivative minus the trace on the two faces normal to p).
Moving both derivatives of grad div onto the basis and testing functions is
one integration by parts on each side.

Dimension reduction (the paper reduces the singular volume-volume integrals
dimension by dimension, Sec. III-C; this is our own route to the same
numbers): every integrand is a product over the three axes of 1-D weights, so
each pair of 1-D integrals over u_i, v_i collapses to one integral over
w_i = u_i - v_i against the correlation of the two 1-D weights.  Correlations
of densities are piecewise polynomials on [-Delta, 0] and [0, Delta];
correlations involving the face deltas are densities on a half interval or
point masses at {-Delta, 0, Delta}.  Each block entry is then a sum of 3-D
(or, with a point mass on one axis, 2-D) integrals of g times a polynomial
over boxes whose corners lie on the lattice Delta * Z.  The only singular
point, w = -d * Delta, is therefore either a box corner (handled by Duffy's
pyramid/triangle split, which cancels the 1/r) or at least one box width away
(plain tensor Gauss-Legendre, order chosen by distance).

Nothing here assumes the symmetries of T; the tests check them.
"""
import numpy as np

from . import physics

_KIND_CACHE = {}


def _gl01(n):
    """Gauss-Legendre nodes/weights on [0, 1]."""
    if n not in _KIND_CACHE:
        x, w = np.polynomial.legendre.leggauss(n)
        _KIND_CACHE[n] = (0.5 * (x + 1.0), 0.5 * w)
    return _KIND_CACHE[n]


# ---------------------------------------------------------------------------
# 1-D measures along one axis.  kinds:
#   '1'  : factor 1 on the voxel
#   't'  : factor t/D on the voxel (t = local coordinate in [-D/2, D/2])
#   'D1' : distributional derivative of 1 restricted to the voxel
#          = delta(t + D/2) - delta(t - D/2)
#   'Dt' : derivative of (t/D) restricted to the voxel
#          = 1/D - 1/2 delta(t - D/2) - 1/2 delta(t + D/2)
# atoms: ('f', c0, c1): density c0 + c1 t on [-D/2, D/2]
#        ('p', s, weight): point mass at t = s D/2, s in {-1, +1}
# ---------------------------------------------------------------------------
def _measure(kind, D):
    if kind == '1':
        return [('f', 1.0, 0.0)]
    if kind == 't':
        return [('f', 0.0, 1.0 / D)]
    if kind == 'D1':
        return [('p', -1, 1.0), ('p', +1, -1.0)]
    if kind == 'Dt':
        return [('f', 1.0 / D, 0.0), ('p', -1, -0.5), ('p', +1, -0.5)]
    raise ValueError(kind)


def _correlate(mu, nu, D):
    """Correlation of a test measure mu(u) and a basis measure nu(v) along one
    axis, as atoms in w = u - v.

    Returns a list of (geom, f) where geom = ('I', lo) means a density on
    [lo, lo + 2] * D/2 given by f, and geom = ('P', c) means a point mass f (a
    float) at w = c * D/2.  Densities are returned as hashable keys that
    _density evaluates, so equal densities are evaluated once per node set.
    """
    out = []
    for A in mu:
        for B in nu:
            if A[0] == 'f' and B[0] == 'f':
                key = ('ff', A[1], A[2], B[1], B[2], D)
                out.append((('I', -2), key))
                out.append((('I', 0), key))
            elif A[0] == 'p' and B[0] == 'f':
                out.append((('I', A[1] - 1), ('pf', A[1], A[2], B[1], B[2], D)))
            elif A[0] == 'f' and B[0] == 'p':
                out.append((('I', -1 - B[1]), ('fp', A[1], A[2], B[1], B[2], D)))
            else:
                out.append((('P', A[1] - B[1]), A[2] * B[2]))
    return out


def _density(key, w):
    """Evaluate a correlation density (see _correlate) at points w."""
    kind, c1, c2, c3, c4, D = key
    h = 0.5 * D
    if kind == 'ff':
        # int a(w + v) b(v) dv over the overlap of the two voxels, with
        # a = c1 + c2 t and b = c3 + c4 t (3-point Gauss is exact here)
        lo = np.maximum(-h, -h - w)
        hi = np.minimum(h, h - w)
        xs, ws = _gl01(3)
        v = lo[..., None] + (hi - lo)[..., None] * xs
        val = (c1 + c2 * (v + w[..., None])) * (c3 + c4 * v)
        return (val * ws).sum(-1) * (hi - lo)
    if kind == 'pf':
        # point mass c2 at u0 = c1 h against density b = c3 + c4 t: b(u0 - w)
        return c2 * (c3 + c4 * (c1 * h - w))
    if kind == 'fp':
        # density a = c1 + c2 t against point mass c4 at v0 = c3 h: a(w + v0)
        return c4 * (c1 + c2 * (w + c3 * h))
    raise ValueError(kind)


def _scalar_kind(l, axis):
    """1-D factor of the scalar basis N^l along an axis (eq. 20)."""
    return 't' if l == axis + 2 else '1'


def _entry_terms(Delta, k0, part='N'):
    """All integral terms of the 144 entries, grouped by box geometry.

    part = 'N': k0^2 delta_pq S - C (the Gram term is added separately);
    part = 'S': S^{ll'} alone, stored in the p = q = x entries;
    part = 'C': C^{pl,ql'} alone;
    part = 'K': the curl operator, < f^{pl}, curl S f^{ql'} > =
    sum_k eps_{pkq} < N^l, S D_k N^{l'} > (the derivative of g moved onto the
    basis function by parts; eps the Levi-Civita symbol).
    Returns dict geom -> list of (entry, coef, atoms) with entry = 12 a + b,
    geom a 3-tuple of per-axis geometries and atoms the per-axis density keys
    or point weights (floats).
    """
    groups = {}
    for p in range(3):
        for l in range(1, 5):
            a = 4 * p + l - 1
            for q in range(3):
                for lp in range(1, 5):
                    b = 4 * q + lp - 1
                    terms = []
                    if part == 'S' and not (p == 0 and q == 0):
                        continue
                    if (part == 'N' and p == q and k0 != 0.0) or part == 'S':
                        # k0^2 S^{ll'}
                        kt = [_scalar_kind(l, i) for i in range(3)]
                        kb = [_scalar_kind(lp, i) for i in range(3)]
                        terms.append((k0 * k0 if part == 'N' else 1.0, kt, kb))
                    if part in ('N', 'C'):
                        # - C^{pl,ql'}: derivative along p on the test side,
                        # along q on the basis side
                        kt = [_scalar_kind(l, i) for i in range(3)]
                        kb = [_scalar_kind(lp, i) for i in range(3)]
                        kt[p] = 'D' + kt[p]
                        kb[q] = 'D' + kb[q]
                        terms.append((-1.0 if part == 'N' else 1.0, kt, kb))
                    if part == 'K' and p != q:
                        k = 3 - p - q                       # the third axis
                        eps = 1.0 if (p, k, q) in ((0, 1, 2), (1, 2, 0), (2, 0, 1)) else -1.0
                        kt = [_scalar_kind(l, i) for i in range(3)]
                        kb = [_scalar_kind(lp, i) for i in range(3)]
                        kb[k] = 'D' + kb[k]
                        terms.append((eps, kt, kb))
                    for coef, kt, kb in terms:
                        per_axis = [_correlate(_measure(kt[i], Delta[i]), _measure(kb[i], Delta[i]), Delta[i])
                                    for i in range(3)]
                        for ax in per_axis[0]:
                            for ay in per_axis[1]:
                                for az in per_axis[2]:
                                    geom = (ax[0], ay[0], az[0])
                                    npts = sum(g[0] == 'P' for g in geom)
                                    if npts > 1:
                                        raise AssertionError("two point-mass axes cannot occur")
                                    groups.setdefault(geom, []).append(
                                        (12 * a + b, coef, (ax[1], ay[1], az[1])))
    return groups


def _green(r, k0):
    return np.exp(-1j * k0 * r) / (4.0 * np.pi * r)


def _gauss_nodes(geom, Delta, n):
    """Tensor Gauss-Legendre nodes (physical w) and weights for a box."""
    xs, ws = _gl01(n)
    axes_pts, axes_w = [], []
    for i in range(3):
        h = 0.5 * Delta[i]
        if geom[i][0] == 'I':
            lo = geom[i][1] * h
            axes_pts.append(lo + 2 * h * xs)
            axes_w.append(2 * h * ws)
        else:
            axes_pts.append(np.array([geom[i][1] * h]))
            axes_w.append(np.array([1.0]))
    W = np.stack(np.meshgrid(*axes_pts, indexing='ij'), -1).reshape(-1, 3)
    wq = np.einsum('i,j,k->ijk', *axes_w).reshape(-1)
    return W, wq


def _duffy_nodes(geom, Delta, corner_codes, n):
    """Nodes for a box whose corner (per-axis codes) is the singular point.

    The box is mapped to the unit cube (or square) with the singular corner at
    the origin and split into pyramids (triangles) with apex at the origin;
    on the pyramid whose base is the face xi_k = 1 we use xi_k = s,
    xi_j = s t_j, with Jacobian s^(dim-1), which cancels the 1/r of g.
    """
    xs, ws = _gl01(n)
    dims = [i for i in range(3) if geom[i][0] == 'I']
    dim = len(dims)
    origin = np.zeros(3)
    sgnL = np.zeros(3)
    for i in range(3):
        h = 0.5 * Delta[i]
        if geom[i][0] == 'I':
            lo = geom[i][1]
            origin[i] = corner_codes[i] * h
            sgnL[i] = (2 * h) if corner_codes[i] == lo else -(2 * h)
        else:
            origin[i] = geom[i][1] * h
    nodes, weights = [], []
    grids = np.meshgrid(*([xs] * dim), indexing='ij')
    wgrid = np.ones_like(grids[0])
    for g_ in np.meshgrid(*([ws] * dim), indexing='ij'):
        wgrid = wgrid * g_
    s = grids[0].ravel()
    ts = [g.ravel() for g in grids[1:]]
    wflat = wgrid.ravel()
    for k in range(dim):
        xi = np.zeros((s.size, dim))
        xi[:, k] = s
        others = [j for j in range(dim) if j != k]
        for j, t in zip(others, ts):
            xi[:, j] = s * t
        W = np.tile(origin, (s.size, 1))
        for jj, i in enumerate(dims):
            W[:, i] += sgnL[i] * xi[:, jj]
        jac = s ** (dim - 1) * np.prod([abs(sgnL[i]) for i in dims])
        nodes.append(W)
        weights.append(wflat * jac)
    return np.concatenate(nodes), np.concatenate(weights)


def _density_matrix(terms, W):
    """R[node, entry] = sum over the geometry's terms of coef * prod of the
    per-axis densities (or point weights) at the nodes."""
    R = np.zeros((W.shape[0], 144), dtype=np.float64)
    cache = {}
    for entry, coef, atoms in terms:
        val = np.full(W.shape[0], coef)
        for i in range(3):
            at = atoms[i]
            if isinstance(at, tuple):
                key = (at, i)
                if key not in cache:
                    cache[key] = _density(at, W[:, i])
                val = val * cache[key]
            else:
                val = val * at
        R[:, entry] += val
    return R


def _order_for(dinf):
    if dinf <= 2:
        return 16
    if dinf <= 4:
        return 10
    if dinf <= 8:
        return 7
    return 5


def galerkin_blocks(dlist, Delta, k0, duffy_order=14, order_scale=1.0, part='N'):
    """T(d) for each integer offset d in dlist (shape [n, 3]), as [n, 12, 12]
    complex128 (Sec. III-B/C, eq. 25a, 26, 33, 42).

    Delta = (dx, dy, dz) in metres, k0 in 1/m.  part = 'S' returns the scalar
    blocks S^{ll'} as [n, 4, 4]; part = 'C' the charge blocks C as [n, 12, 12];
    part = 'K' the blocks K^{pl,ql'}(d) = < f_m^{pl}, curl S f_n^{ql'} > of
    the magnetic operator (eq. 8b, 25b) as [n, 12, 12].
    """
    dlist = np.atleast_2d(np.asarray(dlist, dtype=np.int64))
    Delta = tuple(float(v) for v in Delta)
    groups = _entry_terms(Delta, float(k0), part)
    out = np.zeros((dlist.shape[0], 144), dtype=np.complex128)
    dinf = np.abs(dlist).max(axis=1)
    near = np.where(dinf <= 1)[0]
    far = np.where(dinf > 1)[0]
    Dvec = np.array(Delta)

    # offsets at least one voxel apart: no singular corner anywhere
    bands = {}
    for idx in far:
        n = max(3, int(round(_order_for(dinf[idx]) * order_scale)))
        bands.setdefault(n, []).append(idx)
    for n, idxs in bands.items():
        idxs = np.array(idxs)
        off = dlist[idxs] * Dvec
        for geom, terms in groups.items():
            W, wq = _gauss_nodes(geom, Delta, n)
            R = _density_matrix(terms, W) * wq[:, None]
            r = np.linalg.norm(off[:, None, :] + W[None, :, :], axis=-1)
            out[idxs] += _green(r, k0) @ R

    # touching or coincident voxels: Duffy where the singular point is a corner
    nnear = max(3, int(round(16 * order_scale)))
    for idx in near:
        d = dlist[idx]
        wstar = -2 * d                     # singular point in units of D/2
        for geom, terms in groups.items():
            touch = True
            for i in range(3):
                if geom[i][0] == 'P':
                    touch &= (geom[i][1] == wstar[i])
                else:
                    touch &= (wstar[i] in (geom[i][1], geom[i][1] + 2))
            if touch:
                W, wq = _duffy_nodes(geom, Delta, wstar, duffy_order)
            else:
                W, wq = _gauss_nodes(geom, Delta, nnear)
            R = _density_matrix(terms, W) * wq[:, None]
            r = np.linalg.norm(d * Dvec + W, axis=-1)
            out[idx] += _green(r, k0) @ R

    # identity part of N at d = 0: the Gram matrix (eq. 26, 33)
    out = out.reshape(-1, 12, 12)
    if part == 'S':
        return out[:, :4, :4].copy()
    if part == 'N':
        G = physics.gram_vector(*Delta)
        for idx in np.where(dinf == 0)[0]:
            out[idx] += np.diag(G)
    return out


def toeplitz_full(N, Delta, k0, **kw):
    """All blocks T(d) for d in (-N, N)^3, as [12, 12, 2Nx-1, 2Ny-1, 2Nz-1]
    with index d_i + N_i - 1 (eq. 42: the block depends on m - n only)."""
    Nx, Ny, Nz = N
    dx = np.arange(-Nx + 1, Nx)
    dy = np.arange(-Ny + 1, Ny)
    dz = np.arange(-Nz + 1, Nz)
    D = np.stack(np.meshgrid(dx, dy, dz, indexing='ij'), -1).reshape(-1, 3)
    T = galerkin_blocks(D, Delta, k0, **kw)
    return T.reshape(2 * Nx - 1, 2 * Ny - 1, 2 * Nz - 1, 12, 12).transpose(3, 4, 0, 1, 2).copy()


def toeplitz_octant(N, Delta, k0, **kw):
    """Blocks T(d) for d in [0, N)^3 only (the Toeplitz-defining tensors of
    eq. 43), as [12, 12, Nx, Ny, Nz]."""
    Nx, Ny, Nz = N
    D = np.stack(np.meshgrid(np.arange(Nx), np.arange(Ny), np.arange(Nz), indexing='ij'), -1).reshape(-1, 3)
    T = galerkin_blocks(D, Delta, k0, **kw)
    return T.reshape(Nx, Ny, Nz, 12, 12).transpose(3, 4, 0, 1, 2).copy()
