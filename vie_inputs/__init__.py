"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle
checks.  Holds none of the method's arithmetic: only geometry of phantoms,
material draws, source positions and random vectors.

Every generator takes an explicit seed and uses numpy's PCG64, so the same
seed gives the same bytes on every machine.

Grid convention: the box is centred at the origin; voxel centres at
(n_i - (N_i - 1)/2) * Delta_i.  Arrays are indexed [ix, iy, iz].

Workload recipes (stand-ins for the body models of the paper's experiments,
which are not available):

* ``sphere``: homogeneous sphere, a voxel is inside when its centre is within
  the radius (Sec. V-A geometry, scaled down).
* ``ellipsoid_phantom``: a body ellipsoid (semi-axes 0.45 L_i) of class 0 and
  16 axis-aligned ellipsoids (centres inside the body, semi-axes
  U[0.08, 0.30] L_min, class U{1..n-1}) painted in order and clipped to the
  body; per-class eps' ~ U[5, 80], sigma ~ U[0.05, 2] S/m by default.
* ``layered_phantom``: body ellipsoid with semi-axes (0.40, 0.40, 0.45) L and
  n equal-thickness ellipsoidal shells as classes; eps' ~ U[5, 80],
  sigma ~ U[0.02, 2] S/m.
* ``magnetic_phantom``: the ellipsoid phantom with a per-class permeability
  mu' ~ U[1, 3], mu'' ~ U[0, 0.5] (the J-M formulation's workload; tissue
  is non-magnetic, so this stands in for magnetically loaded materials).
* ``dipoles_on_cylinder``: z-directed unit dipoles (1 A m) at angle U[0, 2 pi)
  and height U[-0.4, 0.4] L_z on a cylinder about the z axis.
"""
import numpy as np

BASE_SEED = 190202196


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def centres(N, Delta):
    return [(np.arange(N[i]) - 0.5 * (N[i] - 1)) * Delta[i] for i in range(3)]


def _grid(N, Delta):
    cx, cy, cz = centres(N, Delta)
    return np.meshgrid(cx, cy, cz, indexing='ij')


def sphere(N, Delta, radius, eps_re, sigma):
    """(eps', sigma) maps [Nx, Ny, Nz]; air (1, 0) outside the sphere."""
    X, Y, Z = _grid(N, Delta)
    inside = X ** 2 + Y ** 2 + Z ** 2 <= radius ** 2
    e = np.where(inside, float(eps_re), 1.0)
    s = np.where(inside, float(sigma), 0.0)
    return e, s


def ellipsoid_phantom(N, Delta, seed, n_classes=6, n_blobs=16,
                      eps_range=(5.0, 80.0), sigma_range=(0.05, 2.0)):
    g = rng(seed)
    eps_c = g.uniform(*eps_range, size=n_classes)
    sig_c = g.uniform(*sigma_range, size=n_classes)
    L = np.array([N[i] * Delta[i] for i in range(3)])
    X, Y, Z = _grid(N, Delta)
    ax = 0.45 * L
    body = (X / ax[0]) ** 2 + (Y / ax[1]) ** 2 + (Z / ax[2]) ** 2 <= 1.0
    cls = np.where(body, 0, -1)
    for _ in range(n_blobs):
        while True:
            c = g.uniform(-ax, ax)
            if np.sum((c / ax) ** 2) <= 1.0:
                break
        semi = g.uniform(0.08, 0.30, size=3) * L.min()
        k = int(g.integers(1, n_classes))
        blob = ((X - c[0]) / semi[0]) ** 2 + ((Y - c[1]) / semi[1]) ** 2 + ((Z - c[2]) / semi[2]) ** 2 <= 1.0
        cls = np.where(blob & body, k, cls)
    e = np.where(cls >= 0, eps_c[np.maximum(cls, 0)], 1.0)
    s = np.where(cls >= 0, sig_c[np.maximum(cls, 0)], 0.0)
    return e, s


def magnetic_phantom(N, Delta, seed, mu_range=(1.0, 3.0), mu_loss_range=(0.0, 0.5), **kw):
    """The ellipsoid phantom of the same seed (identical eps', sigma) with a
    permeability per class drawn after it: mu' ~ U[1, 3], mu'' ~ U[0, 0.5]
    in the body, (1, 0) in air.  Returns (eps', sigma, mu', mu'')."""
    n_classes = kw.get("n_classes", 6)
    e, s = ellipsoid_phantom(N, Delta, seed, **kw)
    # replay the class map: the same draws in the same order
    g = rng(seed)
    g.uniform(0, 1, size=n_classes)
    g.uniform(0, 1, size=n_classes)
    L = np.array([N[i] * Delta[i] for i in range(3)])
    X, Y, Z = _grid(N, Delta)
    ax = 0.45 * L
    body = (X / ax[0]) ** 2 + (Y / ax[1]) ** 2 + (Z / ax[2]) ** 2 <= 1.0
    cls = np.where(body, 0, -1)
    for _ in range(kw.get("n_blobs", 16)):
        while True:
            c = g.uniform(-ax, ax)
            if np.sum((c / ax) ** 2) <= 1.0:
                break
        semi = g.uniform(0.08, 0.30, size=3) * L.min()
        k = int(g.integers(1, n_classes))
        blob = ((X - c[0]) / semi[0]) ** 2 + ((Y - c[1]) / semi[1]) ** 2 + ((Z - c[2]) / semi[2]) ** 2 <= 1.0
        cls = np.where(blob & body, k, cls)
    mu_c = g.uniform(*mu_range, size=n_classes)
    mul_c = g.uniform(*mu_loss_range, size=n_classes)
    mre = np.where(cls >= 0, mu_c[np.maximum(cls, 0)], 1.0)
    mim = np.where(cls >= 0, mul_c[np.maximum(cls, 0)], 0.0)
    return e, s, mre, mim


def layered_phantom(N, Delta, seed, n_classes=10, eps_range=(5.0, 80.0), sigma_range=(0.02, 2.0)):
    g = rng(seed)
    eps_c = g.uniform(*eps_range, size=n_classes)
    sig_c = g.uniform(*sigma_range, size=n_classes)
    L = np.array([N[i] * Delta[i] for i in range(3)])
    X, Y, Z = _grid(N, Delta)
    ax = np.array([0.40, 0.40, 0.45]) * L
    rho = np.sqrt((X / ax[0]) ** 2 + (Y / ax[1]) ** 2 + (Z / ax[2]) ** 2)
    body = rho <= 1.0
    cls = np.minimum(n_classes - 1, np.floor(n_classes * (1.0 - rho)).astype(int))
    e = np.where(body, eps_c[np.clip(cls, 0, n_classes - 1)], 1.0)
    s = np.where(body, sig_c[np.clip(cls, 0, n_classes - 1)], 0.0)
    return e, s


def dipoles_on_cylinder(seed, n, radius, Lz):
    g = rng(seed)
    ang = g.uniform(0.0, 2 * np.pi, size=n)
    z = g.uniform(-0.4 * Lz, 0.4 * Lz, size=n)
    pos = np.stack([radius * np.cos(ang), radius * np.sin(ang), z], 1)
    mom = np.tile(np.array([0.0, 0.0, 1.0]), (n, 1))
    return pos, mom


def dipole_ring(n, ax, ay):
    """n z-directed dipoles at angles 2 pi k / n on an ellipse in the z = 0 plane."""
    ang = 2 * np.pi * np.arange(n) / n
    pos = np.stack([ax * np.cos(ang), ay * np.sin(ang), np.zeros(n)], 1)
    mom = np.tile(np.array([0.0, 0.0, 1.0]), (n, 1))
    return pos, mom


def complex_normal(seed, shape):
    """CN(0, 1) samples (independent real and imaginary parts of variance 1/2)."""
    g = rng(seed)
    return (g.standard_normal(shape) + 1j * g.standard_normal(shape)) / np.sqrt(2.0)


def random_blocks(seed, N):
    """Random unique block tensors [60, Nx, Ny, Nz] complex128 (offsets d >= 0),
    for exercising the operator product on grids where the physical blocks are
    too slow to compute on the CPU."""
    return complex_normal(seed, (60,) + tuple(N))
