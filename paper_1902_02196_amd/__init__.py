"""MI355X volume-integral-equation library (PWL current-based VIE).

Thin ctypes binding of the C ABI in include/vie.h: argument marshalling only,
every step of the computation runs in the HIP library ``libvie.so``.  PyTorch
supplies device memory and streams.  Importing fails loudly when the library
has not been built (``python paper_1902_02196_amd/build.py``); there is no
CPU fallback.

Array layout: vectors of unknowns are torch tensors of shape
(nrhs, nc, Nz, Ny, Nx), complex64 or complex128, on the GPU.  PWL basis
(nc = 12, the default): unknown index a = 4 p + (l - 1) with p the field
component and l the scalar basis (1 pulse, 2..4 linear in x, y, z).  PWC
basis (nc = 3, ``Context.set_basis(3)``): unknown index p, the pulse
coefficients alone.  Per-voxel arrays are (Nz, Ny, Nx).
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvie.so")

VIE_OK, VIE_EINVAL, VIE_ENOMEM, VIE_EDEVICE, VIE_ENOCONV, VIE_ENAN, VIE_ESTATE = 0, -1, -2, -3, -4, -5, -6
C64, C128 = 0, 1
OP_PREC, OP_A, OP_N = 0, 1, 2
SOLVE_FP64, SOLVE_FP32_IR = 0, 1
KERNELS = ("fft_z_fwd", "fft_y_fwd", "block", "fft_y_inv", "fft_z_inv", "gs_dot", "gs_update", "gs_pair")

if not os.path.exists(LIB_PATH):
    raise ImportError("libvie.so is not built; run `python paper_1902_02196_amd/build.py` (needs hipcc)")
_lib = ctypes.CDLL(LIB_PATH)

_vp = ctypes.c_void_p
_i = ctypes.c_int
_d = ctypes.c_double
_dp = ctypes.POINTER(ctypes.c_double)


class SolveOpts(ctypes.Structure):
    _fields_ = [("mode", _i), ("restart", _i), ("max_outer", _i), ("tol", _d), ("inner_tol", _d),
                ("max_refine", _i), ("reorth", _i), ("use_x0", _i),
                ("graph", _i), ("sync_steps", _i), ("s_step", _i)]


class SolveStats(ctypes.Structure):
    _fields_ = [("converged", _i), ("iterations", _i), ("restarts", _i), ("refinements", _i),
                ("matvecs_c64", _i), ("matvecs_c128", _i), ("rel_residual", _d), ("seconds", _d)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class TuckerInfo(ctypes.Structure):
    _fields_ = [("ranks", (_i * 3) * 60), ("rel_error", _d * 60), ("max_rel_error", _d),
                ("bytes_dense", ctypes.c_size_t), ("bytes_compressed", ctypes.c_size_t), ("seconds", _d)]

    def as_dict(self):
        return {"ranks": np.array([[self.ranks[e][i] for i in range(3)] for e in range(60)]),
                "rel_error": np.array(self.rel_error[:]), "max_rel_error": self.max_rel_error,
                "bytes_dense": self.bytes_dense, "bytes_compressed": self.bytes_compressed, "seconds": self.seconds}


class Request(ctypes.Structure):
    _fields_ = [("nx", _i), ("ny", _i), ("nz", _i), ("dx", _d), ("dy", _d), ("dz", _d), ("freq_hz", _d),
                ("eps_re", _dp), ("sigma", _dp), ("nrhs", _i), ("pos", _dp), ("moment", _dp), ("mode", _i),
                ("tol", _d), ("restart", _i), ("x_out", _dp), ("p_abs_out", _dp), ("basis", _i)]


class RequestInfo(ctypes.Structure):
    _fields_ = [("done", _i), ("status", _i), ("t_arrival", _d), ("t_start", _d), ("t_end", _d),
                ("footprint", ctypes.c_size_t), ("iterations", _i), ("rel_residual", _d),
                ("message", ctypes.c_char * 192), ("operator_cached", _i)]


class ServingStats(ctypes.Structure):
    _fields_ = [("completed", _i), ("queued", _i), ("running", _i), ("peak_running", _i), ("p50_s", _d),
                ("p99_s", _d), ("mean_s", _d), ("makespan_s", _d), ("peak_bytes", ctypes.c_size_t),
                ("operator_hits", ctypes.c_longlong), ("operator_misses", ctypes.c_longlong),
                ("operator_cache_bytes", ctypes.c_size_t), ("oldest_queued_s", _d)]


_sig = {
    "vie_create": (_i, [ctypes.POINTER(_vp), _i, _vp]),
    "vie_destroy": (None, [_vp]),
    "vie_last_error": (ctypes.c_char_p, []),
    "vie_set_stream": (_i, [_vp, _vp]),
    "vie_set_grid": (_i, [_vp, _i, _i, _i, _d, _d, _d, _d, ctypes.POINTER(_i)]),
    "vie_set_toeplitz": (_i, [_vp, _dp]),
    "vie_get_toeplitz": (_i, [_vp, _dp]),
    "vie_set_magnetic_contrast": (_i, [_vp, _dp, _dp, _i]),
    "vie_tucker_compress": (_i, [_vp, _d, ctypes.POINTER(TuckerInfo)]),
    "vie_tucker_reconstruct": (_i, [_vp, _vp]),
    "vie_tucker_expand": (_i, [_vp]),
    "vie_set_contrast": (_i, [_vp, _dp, _dp, _i]),
    "vie_incident_planewave": (_i, [_vp, _dp, _dp, _d, _vp]),
    "vie_incident_dipoles": (_i, [_vp, _i, _dp, _dp, _i, _vp]),
    "vie_rhs_prec": (_i, [_vp, _i, _vp, _vp]),
    "vie_apply": (_i, [_vp, _i, _i, _i, _vp, _vp]),
    "vie_apply_noalloc": (_i, [_vp, _i, _i, _i, _vp, _vp]),
    "vie_default_opts": (None, [ctypes.POINTER(SolveOpts)]),
    "vie_solve": (_i, [_vp, ctypes.POINTER(SolveOpts), _i, _vp, _vp, ctypes.POINTER(SolveStats)]),
    "vie_fields": (_i, [_vp, _i, _vp, _vp]),
    "vie_total_field": (_i, [_vp, _i, _vp, _vp, _vp]),
    "vie_absorbed_power": (_i, [_vp, _i, _vp, _dp]),
    "vie_power_density": (_i, [_vp, _i, _vp, _vp]),
    "vie_copy": (_i, [_vp, _vp, _vp, ctypes.c_longlong]),
    "vie_incident_planewave_h": (_i, [_vp, _dp, _dp, _d, _vp]),
    "vie_incident_dipoles_h": (_i, [_vp, _i, _dp, _dp, _i, _vp]),
    "vie_magnetic_field": (_i, [_vp, _i, _vp, _vp, _vp]),
    "vie_b1plus": (_i, [_vp, _i, _vp, _vp]),
    "vie_magnetic_energy": (_i, [_vp, _i, _vp, _vp, _dp]),
    "vie_get_curl_toeplitz": (_i, [_vp, _dp]),
    "vie_autotune": (_i, [_vp, _i, _i, ctypes.POINTER(_i), _dp]),
    "vie_set_tuning": (_i, [_vp, _i, _i, ctypes.POINTER(_i)]),
    "vie_fft_size": (_i, [_vp, ctypes.POINTER(_i)]),
    "vie_set_basis": (_i, [_vp, _i]),
    "vie_share_grid": (_i, [_vp, _vp]),
    "vie_profile": (_i, [_vp, _i]),
    "vie_profile_read": (_i, [_vp, _i, _dp, ctypes.POINTER(_i), _dp]),
    "vie_server_create": (_i, [ctypes.POINTER(_vp), _i, ctypes.c_size_t, _i]),
    "vie_server_submit": (_i, [_vp, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_longlong)]),
    "vie_server_poll": (_i, [_vp, ctypes.c_longlong, ctypes.POINTER(RequestInfo)]),
    "vie_server_wait": (_i, [_vp]),
    "vie_server_stats": (_i, [_vp, ctypes.c_longlong, ctypes.POINTER(ServingStats)]),
    "vie_server_destroy": (None, [_vp]),
    "vie_server_set_operator_cache": (_i, [_vp, ctypes.c_size_t]),
    "vie_unknowns_bytes_paper": (ctypes.c_size_t, [_i, _i, _i]),
    "vie_unknowns_bytes_basis": (ctypes.c_size_t, [_i, _i, _i, _i]),
    "vie_footprint_bytes": (_i, [_i, _i, _i, _i, _i, _i, ctypes.POINTER(ctypes.c_size_t)]),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_sig)


class VieError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (status %d)" % (msg, code))
        self.code = code


def _check(code):
    if code != VIE_OK:
        raise VieError(code, _lib.vie_last_error().decode())
    return code


def _dptr(a):
    return a.ctypes.data_as(_dp)


def _stream_ptr(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def unknowns_bytes_paper(nx, ny, nz):
    """Unknowns memory as the paper counts it: 12 x 8 N_V x 16 B."""
    return int(_lib.vie_unknowns_bytes_paper(nx, ny, nz))


def unknowns_bytes_basis(nx, ny, nz, ncomp):
    """The same count for ncomp unknowns per voxel (12 PWL, 3 PWC)."""
    return int(_lib.vie_unknowns_bytes_basis(nx, ny, nz, ncomp))


def footprint_bytes(nx, ny, nz, nrhs, mode, restart=50):
    out = ctypes.c_size_t(0)
    _check(_lib.vie_footprint_bytes(nx, ny, nz, nrhs, mode, restart, ctypes.byref(out)))
    return int(out.value)


def default_opts(**kw):
    o = SolveOpts()
    _lib.vie_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def _tensor_ptr(t, dtype=None, shape=None):
    import torch
    if not t.is_cuda:
        raise ValueError("expected a GPU tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError("expected dtype %s, got %s" % (dtype, t.dtype))
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("expected shape %s, got %s" % (tuple(shape), tuple(t.shape)))
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """One grid, operator and contrast on one GPU, ordered on one stream."""

    def __init__(self, device=0, stream=None):
        h = ctypes.c_void_p()
        _check(_lib.vie_create(ctypes.byref(h), device, _stream_ptr(stream)))
        self._h = h
        self.N = None
        self.nc = 12

    def close(self):
        if self._h:
            _lib.vie_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream):
        _check(_lib.vie_set_stream(self._h, _stream_ptr(stream)))

    def set_grid(self, N, Delta, freq_hz, fft_size=None):
        nx, ny, nz = (int(v) for v in N)
        fs = None if fft_size is None else (ctypes.c_int * 3)(*[int(v) for v in fft_size])
        _check(_lib.vie_set_grid(self._h, nx, ny, nz, float(Delta[0]), float(Delta[1]), float(Delta[2]),
                                 float(freq_hz), fs))
        self.N = (nx, ny, nz)

    def set_basis(self, ncomp):
        """12: PWL basis (default); 3: PWC basis (pulse functions alone); 24:
        PWL basis, J-M formulation (electric then magnetic currents)."""
        _check(_lib.vie_set_basis(self._h, int(ncomp)))
        self.nc = int(ncomp)

    def share_grid(self, other):
        """Use other's grid and operator (shared device buffers)."""
        _check(_lib.vie_share_grid(self._h, other._h))
        self.N = other.N

    @property
    def fft_size(self):
        """(M_x, M_y, M_z) of the padded FFT grid."""
        m = (ctypes.c_int * 3)()
        _check(_lib.vie_fft_size(self._h, m))
        return tuple(m)

    @property
    def V(self):
        return self.N[0] * self.N[1] * self.N[2]

    def vec_shape(self, nrhs=1):
        return (nrhs, self.nc, self.N[2], self.N[1], self.N[0])

    def set_toeplitz(self, T_unique):
        """T_unique: complex128 [60, Nz, Ny, Nx] (offsets d >= 0)."""
        a = np.ascontiguousarray(T_unique, dtype=np.complex128)
        assert a.shape == (60, self.N[2], self.N[1], self.N[0])
        _check(_lib.vie_set_toeplitz(self._h, a.view(np.float64).ctypes.data_as(_dp)))

    def get_toeplitz(self):
        a = np.zeros((60, self.N[2], self.N[1], self.N[0]), dtype=np.complex128)
        _check(_lib.vie_get_toeplitz(self._h, a.view(np.float64).ctypes.data_as(_dp)))
        return a

    def set_magnetic_contrast(self, mu_re, mu_im):
        """J-M contexts (set_basis(24)): mu', mu'' as float64 arrays [Nz, Ny, Nx]
        on the host, mu_r = mu' - i mu''."""
        a = np.ascontiguousarray(mu_re, dtype=np.float64)
        b = np.ascontiguousarray(mu_im, dtype=np.float64)
        _check(_lib.vie_set_magnetic_contrast(self._h, _dptr(a), _dptr(b), 0))

    def tucker_compress(self, tol):
        """Tucker-compress the 60 unique tensors to relative tolerance tol;
        returns ranks [60, 3] (x, y, z), per-tensor errors and sizes."""
        info = TuckerInfo()
        _check(_lib.vie_tucker_compress(self._h, float(tol), ctypes.byref(info)))
        return info.as_dict()

    def tucker_reconstruct(self, out):
        """T_hat into out: complex128 GPU tensor [60, Nz, Ny, Nx]."""
        import torch
        _check(_lib.vie_tucker_reconstruct(self._h, _tensor_ptr(out, torch.complex128,
                                                                  (60, self.N[2], self.N[1], self.N[0]))))

    def tucker_expand(self):
        """Rebuild the operator from the compressed form."""
        _check(_lib.vie_tucker_expand(self._h))

    def set_contrast(self, eps_re, sigma):
        """eps', sigma as float64 arrays [Nz, Ny, Nx] (numpy on the host or
        torch tensors on the GPU)."""
        if isinstance(eps_re, np.ndarray):
            e = np.ascontiguousarray(eps_re, dtype=np.float64)
            s = np.ascontiguousarray(sigma, dtype=np.float64)
            _check(_lib.vie_set_contrast(self._h, _dptr(e), _dptr(s), 0))
        else:
            e = ctypes.cast(_tensor_ptr(eps_re), _dp)
            s = ctypes.cast(_tensor_ptr(sigma), _dp)
            _check(_lib.vie_set_contrast(self._h, e, s, 1))

    def incident_planewave(self, out, pol=(1.0, 0.0, 0.0), direction=(0.0, 0.0, 1.0), amp=1.0):
        import torch
        p = np.asarray(pol, dtype=np.float64)
        d = np.asarray(direction, dtype=np.float64)
        _check(_lib.vie_incident_planewave(self._h, _dptr(p), _dptr(d), float(amp),
                                           _tensor_ptr(out, torch.complex128, self.vec_shape(1))))

    def incident_dipoles(self, out, positions, moments, nq=4):
        import torch
        pos = np.ascontiguousarray(positions, dtype=np.float64).reshape(-1, 3)
        mom = np.ascontiguousarray(moments, dtype=np.float64).reshape(-1, 3)
        n = pos.shape[0]
        _check(_lib.vie_incident_dipoles(self._h, n, _dptr(pos), _dptr(mom), int(nq),
                                         _tensor_ptr(out, torch.complex128, self.vec_shape(n))))

    def rhs_prec(self, e_t, out):
        import torch
        n = e_t.shape[0]
        _check(_lib.vie_rhs_prec(self._h, n, _tensor_ptr(e_t, torch.complex128, self.vec_shape(n)),
                                 _tensor_ptr(out, torch.complex128, self.vec_shape(n))))

    def apply(self, x, y, op=OP_PREC):
        import torch
        prec = {torch.complex64: C64, torch.complex128: C128}[x.dtype]
        n = x.shape[0]
        _check(_lib.vie_apply(self._h, op, prec, n, _tensor_ptr(x, x.dtype, self.vec_shape(n)),
                              _tensor_ptr(y, x.dtype, self.vec_shape(n))))

    def apply_noalloc(self, x, y, op=OP_PREC):
        """As apply, with the intermediates in the library's fixed per-device
        workspace (vie_apply_noalloc: no device allocation)."""
        import torch
        prec = {torch.complex64: C64, torch.complex128: C128}[x.dtype]
        n = x.shape[0]
        _check(_lib.vie_apply_noalloc(self._h, op, prec, n, _tensor_ptr(x, x.dtype, self.vec_shape(n)),
                                      _tensor_ptr(y, x.dtype, self.vec_shape(n))))

    def solve(self, e_t, x, opts=None, **kw):
        import torch
        o = opts if opts is not None else default_opts(**kw)
        n = e_t.shape[0]
        st = (SolveStats * n)()
        code = _lib.vie_solve(self._h, ctypes.byref(o), n, _tensor_ptr(e_t, torch.complex128, self.vec_shape(n)),
                              _tensor_ptr(x, torch.complex128, self.vec_shape(n)), st)
        if code not in (VIE_OK, VIE_ENOCONV):
            _check(code)
        return code, [s.as_dict() for s in st]

    def fields(self, x, out):
        import torch
        n = x.shape[0]
        _check(_lib.vie_fields(self._h, n, _tensor_ptr(x, torch.complex128, self.vec_shape(n)),
                               _tensor_ptr(out, torch.complex128, self.vec_shape(n))))

    def total_field(self, e_t, x, out):
        """Total field coefficients in the whole box (one operator product)."""
        import torch
        n = x.shape[0]
        _check(_lib.vie_total_field(self._h, n, _tensor_ptr(e_t, torch.complex128, self.vec_shape(n)),
                                    _tensor_ptr(x, torch.complex128, self.vec_shape(n)),
                                    _tensor_ptr(out, torch.complex128, self.vec_shape(n))))

    def incident_planewave_h(self, out, pol=(1.0, 0.0, 0.0), direction=(0.0, 0.0, 1.0), amp=1.0):
        """Tested incident magnetic field of the plane wave (1 / eta0 dir x E)."""
        import torch
        p = np.asarray(pol, dtype=np.float64)
        d = np.asarray(direction, dtype=np.float64)
        _check(_lib.vie_incident_planewave_h(self._h, _dptr(p), _dptr(d), float(amp),
                                             _tensor_ptr(out, torch.complex128, self.vec_shape(1))))

    def incident_dipoles_h(self, out, positions, moments, nq=4):
        import torch
        pos = np.ascontiguousarray(positions, dtype=np.float64).reshape(-1, 3)
        mom = np.ascontiguousarray(moments, dtype=np.float64).reshape(-1, 3)
        n = pos.shape[0]
        _check(_lib.vie_incident_dipoles_h(self._h, n, _dptr(pos), _dptr(mom), int(nq),
                                           _tensor_ptr(out, torch.complex128, self.vec_shape(n))))

    def magnetic_field(self, h_t, x, out):
        """h = G^-1 (h_t + K x): total magnetic field coefficients (curl operator)."""
        import torch
        n = x.shape[0]
        _check(_lib.vie_magnetic_field(self._h, n, _tensor_ptr(h_t, torch.complex128, self.vec_shape(n)),
                                       _tensor_ptr(x, torch.complex128, self.vec_shape(n)),
                                       _tensor_ptr(out, torch.complex128, self.vec_shape(n))))

    def b1plus(self, h, out):
        """b1+ = mu0 (h_x + i h_y) per scalar basis: out (nrhs, 4, Nz, Ny, Nx)."""
        import torch
        n = h.shape[0]
        _check(_lib.vie_b1plus(self._h, n, _tensor_ptr(h, torch.complex128, self.vec_shape(n)),
                               _tensor_ptr(out, torch.complex128, (n, 4, self.N[2], self.N[1], self.N[0]))))

    def magnetic_energy(self, h, density_out=None):
        """W_m over the body per right-hand side (host array); the voxel
        energy density into density_out (nrhs, Nz, Ny, Nx) float64 if given."""
        import torch
        n = h.shape[0]
        W = np.zeros(n)
        dens = None if density_out is None else ctypes.cast(
            _tensor_ptr(density_out, torch.float64, (n, self.N[2], self.N[1], self.N[0])), _vp)
        _check(_lib.vie_magnetic_energy(self._h, n, _tensor_ptr(h, torch.complex128, self.vec_shape(n)), dens,
                                        _dptr(W)))
        return W

    def get_curl_toeplitz(self):
        a = np.zeros((30, self.N[2], self.N[1], self.N[0]), dtype=np.complex128)
        _check(_lib.vie_get_curl_toeplitz(self._h, a.view(np.float64).ctypes.data_as(_dp)))
        return a

    def absorbed_power(self, x):
        import torch
        n = x.shape[0]
        out = np.zeros(n)
        _check(_lib.vie_absorbed_power(self._h, n, _tensor_ptr(x, torch.complex128, self.vec_shape(n)), _dptr(out)))
        return out

    def copy(self, src, dst):
        """Device copy of complex128 tensors (plain streaming kernel)."""
        import torch
        assert src.dtype == torch.complex128 and dst.shape == src.shape
        _check(_lib.vie_copy(self._h, _tensor_ptr(src), _tensor_ptr(dst), src.numel()))

    def autotune(self, precision=C64, nrhs=1):
        """Pick the fastest launch shapes for this grid; returns (choice, ms)."""
        ch = (ctypes.c_int * 4)()
        ms = ctypes.c_double(0)
        _check(_lib.vie_autotune(self._h, precision, nrhs, ch, ctypes.byref(ms)))
        return {"variant": ch[0], "sib_blocks": ch[1], "tile_z": ch[2], "tile_y": ch[3]}, ms.value

    def set_tuning(self, choice, precision=C64, nrhs=1):
        """Install launch shapes (a dict as autotune returns) without timing."""
        ch = (ctypes.c_int * 4)(int(choice["variant"]), int(choice["sib_blocks"]), int(choice["tile_z"]),
                                int(choice["tile_y"]))
        _check(_lib.vie_set_tuning(self._h, precision, nrhs, ch))

    def profile(self, enable=True, every=1):
        """Time launches by class with HIP events (one launch in `every`)."""
        _check(_lib.vie_profile(self._h, int(every) if enable else 0))

    def profile_read(self):
        """{kernel class: (total ms, launches, algorithmic bytes)}"""
        out = {}
        for k, name in enumerate(KERNELS):
            ms, n, b = ctypes.c_double(0), ctypes.c_int(0), ctypes.c_double(0)
            _check(_lib.vie_profile_read(self._h, k, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(b)))
            out[name] = (ms.value, n.value, b.value)
        return out

    def power_density(self, e, out):
        import torch
        n = e.shape[0]
        _check(_lib.vie_power_density(self._h, n, _tensor_ptr(e, torch.complex128, self.vec_shape(n)),
                                      _tensor_ptr(out, torch.float64, (n, self.N[2], self.N[1], self.N[0]))))


class Server:
    """Continuous-batching solve server on one GPU (C++ scheduler and worker
    threads in the library).  Requests are admitted while their device
    footprints fit ``hbm_budget`` bytes and at most ``max_slots`` run at once;
    each runs on its own context and stream.  Results land in host arrays
    owned by this object until :meth:`result` hands them out."""

    def __init__(self, device=0, hbm_budget=64 << 30, max_slots=4):
        h = ctypes.c_void_p()
        _check(_lib.vie_server_create(ctypes.byref(h), int(device), int(hbm_budget), int(max_slots)))
        self._h = h
        self._held = {}

    def close(self):
        if self._h:
            _lib.vie_server_destroy(self._h)
            self._h = None
            self._held.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, N, Delta, freq_hz, eps_re, sigma, positions, moments, mode=SOLVE_FP32_IR, tol=1e-6,
               restart=50, want_x=False, basis=12):
        """Queue one request (nrhs = number of dipoles; basis 12 PWL or 3 PWC); returns its id."""
        nx, ny, nz = (int(v) for v in N)
        e = np.ascontiguousarray(eps_re, dtype=np.float64)
        sg = np.ascontiguousarray(sigma, dtype=np.float64)
        if e.shape != (nz, ny, nx) or sg.shape != (nz, ny, nx):
            raise ValueError("eps_re and sigma must have shape (Nz, Ny, Nx)")
        pos = np.ascontiguousarray(positions, dtype=np.float64).reshape(-1, 3)
        mom = np.ascontiguousarray(moments, dtype=np.float64).reshape(-1, 3)
        if pos.shape != mom.shape:
            raise ValueError("positions and moments differ in length")
        n = pos.shape[0]
        p_abs = np.zeros(n)
        x = np.zeros((n, int(basis), nz, ny, nx), dtype=np.complex128) if want_x else None
        r = Request(nx, ny, nz, float(Delta[0]), float(Delta[1]), float(Delta[2]), float(freq_hz), _dptr(e),
                    _dptr(sg), n, _dptr(pos), _dptr(mom), int(mode), float(tol), int(restart),
                    x.view(np.float64).ctypes.data_as(_dp) if want_x else None, _dptr(p_abs), int(basis))
        rid = ctypes.c_longlong(-1)
        _check(_lib.vie_server_submit(self._h, ctypes.byref(r), ctypes.byref(rid)))
        self._held[rid.value] = (p_abs, x)
        return rid.value

    def poll(self, rid):
        info = RequestInfo()
        _check(_lib.vie_server_poll(self._h, int(rid), ctypes.byref(info)))
        d = {k: getattr(info, k) for k, _ in info._fields_}
        d["message"] = info.message.decode(errors="replace")
        return d

    def result(self, rid):
        """(info, absorbed power per dipole, x or None) of a finished request."""
        info = self.poll(rid)
        if not info["done"]:
            raise VieError(VIE_ESTATE, "request %d is not finished" % rid)
        p_abs, x = self._held[rid]
        return info, p_abs, x

    def wait(self):
        _check(_lib.vie_server_wait(self._h))

    def set_operator_cache(self, nbytes):
        """Device bytes kept for operators of recently used grids (0: off)."""
        _check(_lib.vie_server_set_operator_cache(self._h, int(nbytes)))

    def stats(self, first_id=0):
        st = ServingStats()
        _check(_lib.vie_server_stats(self._h, int(first_id), ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in st._fields_}
