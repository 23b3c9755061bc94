"""Galerkin blocks through the Gaussian representation of the kernel
(TEST INFRASTRUCTURE, see the package docstring).

A second, independent numerical route to the blocks T(d) of the N operator
(Sec. III-B/C, eq. 25a, 32-34, 42), written to pin ``oracle.toeplitz`` where
the singularity of g makes quadrature delicate: touching and coincident
voxels (max |d_i| <= 1), every one of the 144 entries, linear functions and
off-diagonal components included.

The operator split is the one the paper implies (eq. 8a, 10, 13): with
curl curl = grad div - Laplacian and (Laplacian + k0^2) g = -delta,
N = I + k0^2 S + grad div S, whose Galerkin blocks are

    T^{pl,ql'}(d) = delta_{d,0} <f^{pl}, f^{ql'}>
                    + k0^2 delta_pq <N^l, S N^{l'}>(d) - <D_p N^l, S D_q N^{l'}>(d)

with D_p the distributional derivative along p of a function restricted to
its voxel (integration by parts on both sides of grad div).  Each inner
product is a 6-D integral of g(dDelta + u - v) against a product over the
three axes of 1-D measures in u (test side) and v (basis side): densities
(polynomials on the voxel) and, for derivatives, point masses on the faces.

Nothing is split into boxes or mapped around the singular point.  Instead:

* The kernel is expanded in powers of R = |r - r'|,
      exp(-i k0 R) / (4 pi R) = (1 / 4 pi) sum_n (-i k0)^n R^(n-1) / n!,
  which converges fast for the near offsets (k0 R << 1 for voxels well
  below the wavelength, as the method requires).
* Even powers R^(2m) = (w_x^2 + w_y^2 + w_z^2)^m are polynomials: their
  integrals are exact products of 1-D integrals.
* Odd powers R^(2m+1) = R^(2m+2) / R and the static term 1/R use
      1 / R = (2 / sqrt(pi)) int_0^inf exp(-t^2 R^2) dt,
  under which exp(-t^2 R^2) factors over the axes.  For every t the 1-D
  factors are exact: the pair of 1-D measures along an axis is first turned
  into the distribution of w = c + u - v (piecewise polynomial densities and
  point masses, built with exact polynomial arithmetic), then
  int w^j exp(-t^2 w^2) dw over each piece is an incomplete gamma function.
  The remaining integral over t is smooth; with t = exp(s) / L it decays
  exponentially at both ends of the s line, where the trapezoidal rule
  converges geometrically.

Lengths are in metres, k0 in 1/m; unknown index a = 4 p + (l - 1) (eq. 30),
scalar functions N^1 = 1, N^{2,3,4} = (x, y, z - voxel centre) / Delta on
the voxel (eq. 19-22).
"""
import math
from functools import lru_cache

import numpy as np
from numpy.polynomial import polynomial as npoly
from scipy import special

# ---------------------------------------------------------------------------
# 1-D measures on a voxel [-h, h] (h = Delta / 2): ("poly", coefficients in
# the local coordinate, lowest degree first) and point masses (position,
# weight)
# ---------------------------------------------------------------------------


def scalar_factor(l, axis, Delta):
    """1-D factor of the scalar function N^l along an axis: the polynomial
    (in the local coordinate) of eq. 20-22."""
    if l == axis + 2:
        return np.array([0.0, 1.0 / Delta])
    return np.array([1.0])


def plain_measure(poly, Delta):
    return (np.asarray(poly, dtype=np.float64), [])


def derivative_measure(poly, Delta):
    """Distributional derivative of poly * indicator([-h, h]): the interior
    derivative plus poly(-h) delta(t + h) - poly(h) delta(t - h)."""
    h = 0.5 * Delta
    poly = np.asarray(poly, dtype=np.float64)
    dp = np.array([k * poly[k] for k in range(1, poly.size)]) if poly.size > 1 else np.array([0.0])
    return (dp, [(-h, float(npoly.polyval(-h, poly))), (h, -float(npoly.polyval(h, poly)))])


# ---------------------------------------------------------------------------
# distribution of w = c + u - v for u ~ mu (test), v ~ nu (basis)
# ---------------------------------------------------------------------------


def _padd(a, b):
    n = max(len(a), len(b))
    out = np.zeros(n)
    out[:len(a)] += a
    out[:len(b)] += b
    return out


def _shift(poly, c):
    """Coefficients of p(x + c) as a polynomial in x."""
    out = np.zeros(max(len(poly), 1))
    for k, a in enumerate(poly):
        for m in range(k + 1):
            out[m] += a * math.comb(k, m) * c ** (k - m)
    return out


def _compose_linear(biv, alpha, beta):
    """sum_ij biv[i, j] s^i (alpha + beta s)^j as a polynomial in s."""
    out = np.zeros(biv.shape[0] + biv.shape[1])
    for j in range(biv.shape[1]):
        lin = np.array([1.0])
        for _ in range(j):
            lin = np.convolve(lin, [alpha, beta])
        for i in range(biv.shape[0]):
            if biv[i, j] != 0.0:
                term = np.zeros(i + 1)
                term[i] = biv[i, j]
                prod = np.convolve(term, lin)
                out[:len(prod)] += prod
    return out


def pair_distribution(mu, nu, c, Delta):
    """Pieces (lo, hi, polynomial in w) and point masses (w0, weight) of the
    measure of w = c + u - v (u in the test voxel, v in the basis voxel, both
    local coordinates on [-h, h], c the centre offset)."""
    h = 0.5 * Delta
    pa, pts_a = mu
    pb, pts_b = nu
    pieces, masses = [], []
    if np.any(pa) and np.any(pb):
        # a(s + v) b(v) as a bivariate polynomial in (s, v), s = w - c = u - v
        na, nb = len(pa), len(pb)
        biv = np.zeros((na, na + nb))
        for k, ak in enumerate(pa):
            for m in range(k + 1):
                for n_, bn in enumerate(pb):
                    biv[m, k - m + n_] += ak * math.comb(k, m) * bn
        # antiderivative in v
        anti = np.zeros((biv.shape[0], biv.shape[1] + 1))
        for j in range(biv.shape[1]):
            anti[:, j + 1] = biv[:, j] / (j + 1)
        # s in [-2h, 0]: v from -h - s to h;  s in [0, 2h]: v from -h to h - s
        lower = _padd(_compose_linear(anti, h, 0.0), -_compose_linear(anti, -h, -1.0))
        upper = _padd(_compose_linear(anti, h, -1.0), -_compose_linear(anti, -h, 0.0))
        pieces.append((c - 2 * h, c, _shift(lower, -c)))
        pieces.append((c, c + 2 * h, _shift(upper, -c)))
    if np.any(pa):
        for v0, wb in pts_b:
            # u = w - c + v0 in [-h, h]: density wb * a(w - c + v0)
            pieces.append((c - v0 - h, c - v0 + h, wb * _shift(pa, v0 - c)))
    if np.any(pb):
        for u0, wa in pts_a:
            # v = c + u0 - w in [-h, h]: density wa * b(c + u0 - w)
            q = _shift(pb, c + u0)                       # b(x + c + u0) with x = -w
            q = q * ((-1.0) ** np.arange(len(q)))         # b(c + u0 - w)
            pieces.append((c + u0 - h, c + u0 + h, wa * q))
    for u0, wa in pts_a:
        for v0, wb in pts_b:
            masses.append((c + u0 - v0, wa * wb))
    return pieces, masses


# ---------------------------------------------------------------------------
# 1-D factors: exact polynomial moments and Gaussian-weighted moments
# ---------------------------------------------------------------------------


def poly_moment(dist, q):
    """int w^q d(measure)."""
    pieces, masses = dist
    s = 0.0
    for lo, hi, p in pieces:
        for j, cj in enumerate(p):
            if cj != 0.0:
                s += cj * (hi ** (j + q + 1) - lo ** (j + q + 1)) / (j + q + 1)
    for w0, m in masses:
        s += m * w0 ** q
    return s


def _half_moment(p, b, t):
    """int_0^b w^p exp(-t^2 w^2) dw for b >= 0 (arrays t > 0)."""
    a = 0.5 * (p + 1)
    with np.errstate(over='ignore'):   # t^(p+1) beyond the double range: the moment is 0 there
        return special.gammainc(a, (t * b) ** 2) * special.gamma(a) / (2.0 * t ** (p + 1))


def _pos_moment(p, lo, hi, t):
    """int_lo^hi w^p exp(-t^2 w^2) dw for 0 <= lo < hi."""
    a = 0.5 * (p + 1)
    if lo == 0.0:
        return _half_moment(p, hi, t)
    xl, xh = (t * lo) ** 2, (t * hi) ** 2
    lower = special.gammainc(a, xh) - special.gammainc(a, xl)
    upper = special.gammaincc(a, xl) - special.gammaincc(a, xh)
    d = np.where(xl > a, upper, lower)   # the difference that does not cancel
    with np.errstate(over='ignore'):
        return d * special.gamma(a) / (2.0 * t ** (p + 1))


def gauss_moment(p, lo, hi, t):
    """int_lo^hi w^p exp(-t^2 w^2) dw, any lo < hi."""
    if lo >= 0.0:
        return _pos_moment(p, lo, hi, t)
    if hi <= 0.0:
        return (-1.0) ** p * _pos_moment(p, -hi, -lo, t)
    return _half_moment(p, hi, t) + (-1.0) ** p * _half_moment(p, -lo, t)


def gauss_factor(dist, q, t):
    """int w^q exp(-t^2 w^2) d(measure) on the t nodes."""
    pieces, masses = dist
    out = np.zeros_like(t)
    for lo, hi, p in pieces:
        for j, cj in enumerate(p):
            if cj != 0.0:
                out += cj * gauss_moment(j + q, lo, hi, t)
    for w0, m in masses:
        out += m * w0 ** q * np.exp(-(t * w0) ** 2)
    return out


# ---------------------------------------------------------------------------
# t nodes: t = exp(s) / L, trapezoidal rule in s
# ---------------------------------------------------------------------------


def t_nodes(L, step=0.05, s_lo=-36.0, s_hi=34.0):
    s = np.arange(s_lo, s_hi + 0.5 * step, step)
    t = np.exp(s) / L
    return t, step * t   # nodes, weights of dt


def _compositions(m):
    """(a, b, c) >= 0 with a + b + c = m and the multinomial coefficient."""
    for a in range(m + 1):
        for b in range(m + 1 - a):
            c = m - a - b
            yield (a, b, c), math.factorial(m) // (math.factorial(a) * math.factorial(b) * math.factorial(c))


# ---------------------------------------------------------------------------
# blocks
# ---------------------------------------------------------------------------


def _factor_key(deriv, l, axis):
    """The 1-D factor of N^l along an axis, plain or differentiated: one of
    four kinds per side ('one' or 'lin', 'n' or 'd')."""
    return ('d' if deriv else 'n', 'lin' if l == axis + 2 else 'one')


@lru_cache(maxsize=None)
def _dist(key_t, key_b, d, Delta):
    mu_p = np.array([0.0, 1.0 / Delta]) if key_t[1] == 'lin' else np.array([1.0])
    nu_p = np.array([0.0, 1.0 / Delta]) if key_b[1] == 'lin' else np.array([1.0])
    mu = derivative_measure(mu_p, Delta) if key_t[0] == 'd' else plain_measure(mu_p, Delta)
    nu = derivative_measure(nu_p, Delta) if key_b[0] == 'd' else plain_measure(nu_p, Delta)
    return pair_distribution(mu, nu, d * Delta, Delta)


class _Axis:
    """The distribution of w along one axis and its factors on the t nodes
    (cached: only a few distinct factor pairs occur)."""
    cache = {}

    def __init__(self, key_t, key_b, d, Delta, tgrid):
        self.dist = _dist(key_t, key_b, d, Delta)
        self.key = (key_t, key_b, d, Delta, tgrid[2])
        self.t = tgrid[0]

    def gauss(self, q):
        k = self.key + (q,)
        if k not in _Axis.cache:
            _Axis.cache[k] = gauss_factor(self.dist, q, self.t)
        return _Axis.cache[k]

    def poly(self, q):
        return poly_moment(self.dist, q)


def _series_order(k0, rmax):
    if k0 == 0.0:
        return 0
    x = abs(k0) * rmax
    n, term = 0, 1.0
    while term > 1e-18 or n < 2:
        n += 1
        term = x ** n / math.factorial(n)
    return n


def axis_integral(axes, k0, wt, nmax):
    """int int mu(u) nu(v) g(|c + u - v|) from the three per-axis factors,
    g = exp(-i k0 R) / (4 pi R) expanded in powers of R."""
    total = 0.0 + 0.0j
    for n in range(nmax + 1):
        coef = (-1j * k0) ** n / math.factorial(n) / (4.0 * math.pi)
        if n % 2 == 1:
            m = (n - 1) // 2      # R^(2m): a polynomial, exact per axis
            acc = 0.0
            for (a, b, c), mult in _compositions(m):
                acc += mult * axes[0].poly(2 * a) * axes[1].poly(2 * b) * axes[2].poly(2 * c)
            total += coef * acc
        else:
            m = n // 2            # R^(2m - 1) = R^(2m) / R: Gaussian representation of 1/R
            integrand = 0.0
            for (a, b, c), mult in _compositions(m):
                integrand = integrand + mult * axes[0].gauss(2 * a) * axes[1].gauss(2 * b) * axes[2].gauss(2 * c)
            total += coef * (2.0 / math.sqrt(math.pi)) * float(np.dot(integrand, wt))
    return total


def curl_axis_integral(axes, k, k0, t, wt, nmax):
    """int int N^l(u) N^l'(v) d_k g(c + u - v) with the derivative left on
    the kernel (no integration by parts):
        d_k g = -(w_k / 4 pi) sum_n c_n R^(n - 3),
        c_n = (-i k0)^n (1 - n) / n!   (exp(-i k0 R) (1 + i k0 R) in powers of R),
    R^-3 through 1 / R^3 = (4 / sqrt(pi)) int_0^inf t^2 exp(-t^2 R^2) dt, odd
    powers through R^(2m) / R as above, even powers as polynomials; axis k
    carries the extra factor w_k (odd moments)."""
    total = 0.0 + 0.0j
    odd = [1 if i == k else 0 for i in range(3)]
    for n in range(nmax + 1):
        cn = (-1j * k0) ** n * (1 - n) / math.factorial(n)
        if cn == 0:
            continue
        e = n - 3
        if e == -3:
            integrand = axes[0].gauss(odd[0]) * axes[1].gauss(odd[1]) * axes[2].gauss(odd[2])
            val = (4.0 / math.sqrt(math.pi)) * float(np.dot(integrand * t * t, wt))
        elif e % 2 == 0:
            val = 0.0
            for (a, b, c), mult in _compositions(e // 2):
                val += mult * (axes[0].poly(2 * a + odd[0]) * axes[1].poly(2 * b + odd[1]) *
                               axes[2].poly(2 * c + odd[2]))
        else:
            integrand = 0.0
            for (a, b, c), mult in _compositions((e + 1) // 2):
                integrand = integrand + mult * (axes[0].gauss(2 * a + odd[0]) * axes[1].gauss(2 * b + odd[1]) *
                                                 axes[2].gauss(2 * c + odd[2]))
            val = (2.0 / math.sqrt(math.pi)) * float(np.dot(integrand, wt))
        total += -cn * val / (4.0 * math.pi)
    return total


def _levi(p, k, q):
    if (p, k, q) in ((0, 1, 2), (1, 2, 0), (2, 0, 1)):
        return 1.0
    if (p, k, q) in ((0, 2, 1), (2, 1, 0), (1, 0, 2)):
        return -1.0
    return 0.0


def _gram_1d(l, lp, axis, Delta):
    """int over the voxel of the product of the two 1-D factors."""
    h = 0.5 * Delta
    a = np.array([0.0, 1.0 / Delta]) if l == axis + 2 else np.array([1.0])
    b = np.array([0.0, 1.0 / Delta]) if lp == axis + 2 else np.array([1.0])
    p = np.convolve(a, b)
    return sum(c * (h ** (j + 1) - (-h) ** (j + 1)) / (j + 1) for j, c in enumerate(p))


def blocks(dlist, Delta, k0, step=0.05, part='N'):
    """T(d) [n, 12, 12] for integer offsets d (rows of dlist) by the Gaussian
    route.  part = 'N': the whole block (the Gram term of the identity
    included at d = 0); 'S': the scalar blocks <N^l, S N^l'> as [n, 4, 4];
    'C': the charge blocks <D_p N^l, S D_q N^l'> as [n, 12, 12]; 'K': the
    blocks <f^{pl}, curl S f^{ql'}> of the magnetic operator (eq. 8b, 25b),
    sum_k eps_pkq <N^l, S D_k N^l'> (derivative moved onto the basis);
    'Kcurl': the same blocks with the derivative of g kept on the kernel
    (no integration by parts, so no face terms)."""
    dlist = np.atleast_2d(np.asarray(dlist, dtype=np.int64))
    Delta = tuple(float(v) for v in Delta)
    L = max(Delta)
    t, wt = t_nodes(L, step)
    tgrid = (t, wt, (L, step))
    out = []
    for d in dlist:
        d = tuple(int(v) for v in d)
        rmax = float(np.sqrt(sum(((abs(d[i]) + 1) * Delta[i]) ** 2 for i in range(3))))
        nmax = _series_order(float(k0), rmax)

        def integral(der_t, l, der_b, lp):
            axes = [_Axis(_factor_key(der_t == i, l, i), _factor_key(der_b == i, lp, i), d[i], Delta[i], tgrid)
                    for i in range(3)]
            return axis_integral(axes, float(k0), wt, nmax)

        if part in ('K', 'Kcurl'):
            blk = np.zeros((12, 12), dtype=np.complex128)
            Q = {}
            for p in range(3):
                for q in range(3):
                    if p == q:
                        continue
                    k = 3 - p - q
                    for l in range(1, 5):
                        for lp in range(1, 5):
                            if (k, l, lp) not in Q:
                                if part == 'K':
                                    Q[(k, l, lp)] = integral(-1, l, k, lp)
                                else:
                                    axes = [_Axis(_factor_key(False, l, i), _factor_key(False, lp, i), d[i],
                                                  Delta[i], tgrid) for i in range(3)]
                                    Q[(k, l, lp)] = curl_axis_integral(axes, k, float(k0), t, wt, nmax + 1)
                            blk[4 * p + l - 1, 4 * q + lp - 1] = _levi(p, k, q) * Q[(k, l, lp)]
            out.append(blk)
            continue
        if part == 'S':
            S = np.zeros((4, 4), dtype=np.complex128)
            for l in range(1, 5):
                for lp in range(1, 5):
                    S[l - 1, lp - 1] = integral(-1, l, -1, lp)
            out.append(S)
            continue
        blk = np.zeros((12, 12), dtype=np.complex128)
        for p in range(3):
            for l in range(1, 5):
                for q in range(3):
                    for lp in range(1, 5):
                        Cv = integral(p, l, q, lp)     # derivative along p (test), along q (basis)
                        if part == 'C':
                            blk[4 * p + l - 1, 4 * q + lp - 1] = Cv
                            continue
                        v = -Cv
                        if p == q and k0 != 0.0:
                            v += k0 * k0 * integral(-1, l, -1, lp)
                        if p == q and not any(d):
                            v += np.prod([_gram_1d(l, lp, i, Delta[i]) for i in range(3)])
                        blk[4 * p + l - 1, 4 * q + lp - 1] = v
        out.append(blk)
    return np.array(out)
