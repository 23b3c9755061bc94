"""Fields and absorbed power from the solution (TEST INFRASTRUCTURE).

Paper Sec. IV-C and eq. (44); error metrics of Sec. V-C.
x holds the current coefficients x^{pl} [12, Nx, Ny, Nz] (eq. 19, j = c_e chi e).
"""
import numpy as np

from . import physics
from .matvec import direct_N


def fields_from_currents(x, chi, freq_hz):
    """Field coefficients e^{pl} = x^{pl} / (c_e chi) on voxels with chi != 0
    (eq. 6 with the PWC contrast of eq. 23); zero elsewhere."""
    ce = physics.c_e(freq_hz)
    out = np.zeros_like(x)
    m = chi != 0
    out[:, m] = x[:, m] / (ce * chi[m])
    return out


def total_field(T, x, e_t, Delta, freq_hz, Nx_fn=direct_N):
    """Total field coefficients everywhere in the box through one operator
    product (Sec. IV-C): the tested total field G e = e_t + (1/c_e)(N - G) x
    (discrete eq. 'tot_fields' a), divided by the Gram matrix."""
    G = physics.gram_vector(*Delta)[:, None, None, None]
    ce = physics.c_e(freq_hz)
    return e_t / G + (Nx_fn(T, x) / G - x) / ce


def absorbed_power(x, chi, Delta, freq_hz):
    """P_abs = 1/2 Re{ x^* (c_e M_chi)^-1 G x }  (eq. 44), over chi != 0."""
    G = physics.gram_vector(*Delta)[:, None, None, None]
    ce = physics.c_e(freq_hz)
    m = chi != 0
    q = np.zeros(chi.shape, dtype=np.complex128)
    q[m] = 1.0 / (ce * chi[m])
    return 0.5 * float(np.real(np.sum(np.conj(x) * G * x * q[None])))


def power_density(e, sigma):
    """Voxel average of p_abs = 1/2 sigma |e|^2 (Sec. V-C): with the Gram
    weights of eq. 33, 1/2 sigma (sum_p |e^{p1}|^2 + 1/12 sum_{p, l>1} |e^{pl}|^2)."""
    w = np.tile(np.array([1.0, 1.0 / 12, 1.0 / 12, 1.0 / 12]), 3)[:, None, None, None]
    return 0.5 * sigma * np.sum(w * np.abs(e) ** 2, axis=0)


def rel_errors(P, P_ref, p, p_ref, e, e_ref, Delta):
    """error_e1, error_e2, error_e3 of Sec. V-C.  The norm of error_e3 is the
    Gram-weighted (L2 of the field) norm over the voxels given."""
    G = physics.gram_vector(*Delta)[:, None, None, None]
    e1 = abs(P - P_ref) / abs(P_ref)
    e2 = np.sum(np.abs(p - p_ref)) / np.sum(np.abs(p_ref))
    e3 = np.sqrt(np.sum(G * np.abs(e - e_ref) ** 2) / np.sum(G * np.abs(e_ref) ** 2))
    return e1, e2, e3
