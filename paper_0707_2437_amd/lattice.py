"""Python binding of liblbm: one class per C handle, same call names.

Host fields are numpy float64 arrays of shape (ny, nx); populations are
(9, ny, nx). Device variants take torch CUDA (HIP) float64 tensors and pass
their pointers through; torch supplies only device memory and streams.
"""
import ctypes
import sys

import numpy as np

from ._lib import lib

F64, F32, F32S, F16S = 0, 1, 2, 3
DTYPES = {"f64": F64, "f32": F32, "f32s": F32S, "f16s": F16S}
DTYPE_NAMES = {v: k for k, v in DTYPES.items()}

OK, EINVAL, ENOMEM, EDEVICE, ESTATE, ENONFINITE = 0, -1, -2, -3, -4, -5

# lbm_model: the paper's forcing model (Eq. 5) or the altered-equilibrium one
MODEL_FORCING, MODEL_EQUILIBRIUM = 0, 1
XBC_PERIODIC, XBC_INLET_OUTLET = 0, 1


class LBMError(RuntimeError):
    def __init__(self, status, what):
        msg = lib().lbm_strerror(status).decode()
        super().__init__(f"{what}: {msg} ({status})")
        self.status = status


def _check(st, what):
    if st != OK:
        raise LBMError(st, what)
    return st


def _dtype_code(dtype):
    return DTYPES[dtype] if isinstance(dtype, str) else int(dtype)


def footprint_bytes(nx, ny, dtype):
    return lib().lbm_footprint_bytes(int(nx), int(ny), _dtype_code(dtype))


def _host(a, shape):
    if a is None:
        return None
    a = np.asarray(a, dtype=np.float64)
    if a.shape != shape:
        a = np.broadcast_to(a, shape)
    return np.ascontiguousarray(a)


def _hptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _dptr(t, n):
    if t is None:
        return None
    import torch

    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()
            and t.numel() == n):
        raise ValueError("device fields must be contiguous float64 CUDA tensors with nx*ny elements")
    return ctypes.c_void_p(t.data_ptr())


class Lattice:
    """A periodic nx x ny lattice of the variable-speed-of-sound model on the GPU."""

    def __init__(self, nx, ny, tau, c2, dtype="f64", model=MODEL_FORCING):
        self.nx, self.ny, self.tau, self.c2 = int(nx), int(ny), float(tau), float(c2)
        self.dtype = _dtype_code(dtype)
        self._L = lib()
        h = self._L.lbm_create(self.nx, self.ny, self.tau, self.c2, self.dtype)
        if not h:
            raise LBMError(self._L.lbm_last_error(), "lbm_create")
        self._h = ctypes.c_void_p(h)
        self._stream_ref = None
        if model != MODEL_FORCING:
            self.set_model(model)

    def set_model(self, model):
        """lbm_set_model: MODEL_FORCING (Eq. 5) or MODEL_EQUILIBRIUM; before init."""
        _check(self._L.lbm_set_model(self._h, int(model)), "lbm_set_model")
        return self

    def set_x_boundaries(self, mode, amplitude=0.0, period=0.0):
        """lbm_set_x_boundaries: XBC_PERIODIC, or XBC_INLET_OUTLET (Fig. 1:
        rho_in(t) = 1 + amplitude sin(2 pi t / period) at x = 0, rho = 1 at x = nx - 1)."""
        _check(self._L.lbm_set_x_boundaries(self._h, int(mode), float(amplitude), float(period)),
               "lbm_set_x_boundaries")
        return self

    def set_c2_field(self, c2):
        """lbm_set_c2_field: per-site c_e^2 (host array, shape (ny, nx), broadcast
        if smaller), or None to remove the field."""
        c2 = _host(c2, (self.ny, self.nx))
        _check(self._L.lbm_set_c2_field(self._h, _hptr(c2)), "lbm_set_c2_field")
        return self

    def set_c2_field_device(self, c2):
        """lbm_set_c2_field_device: a device FP64 tensor of nx * ny entries
        (row-major), or None; asynchronous on the lattice's stream."""
        _check(self._L.lbm_set_c2_field_device(self._h, _dptr(c2, self.nx * self.ny)), "lbm_set_c2_field_device")
        return self

    # lifetime --------------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            self._L.lbm_destroy(self._h)
            self._h = None

    def __del__(self):
        # At interpreter shutdown the device runtime may already be going
        # away; the process's device memory is released with it, so a handle
        # still open then is left alone (close() it explicitly before exit).
        if not sys.is_finalizing():
            self.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def handle(self):
        return self._h

    # the five calls ----------------------------------------------------------
    def init(self, rho=None, ux=None, uy=None):
        shape = (self.ny, self.nx)
        rho, ux, uy = _host(rho, shape), _host(ux, shape), _host(uy, shape)
        _check(self._L.lbm_init(self._h, _hptr(rho), _hptr(ux), _hptr(uy)), "lbm_init")
        return self

    def init_device(self, rho=None, ux=None, uy=None):
        n = self.nx * self.ny
        _check(self._L.lbm_init_device(self._h, _dptr(rho, n), _dptr(ux, n), _dptr(uy, n)), "lbm_init_device")
        return self

    def step(self, n=1):
        _check(self._L.lbm_step(self._h, int(n)), "lbm_step")
        return self

    def moments(self, fields=True, check=True):
        """(rho, ux, uy, totals) as host arrays; totals = (sum rho, sum rho ux, sum rho uy)."""
        shape = (self.ny, self.nx)
        rho = np.empty(shape) if fields else None
        ux = np.empty(shape) if fields else None
        uy = np.empty(shape) if fields else None
        tot = np.empty(3)
        st = self._L.lbm_moments(self._h, _hptr(rho), _hptr(ux), _hptr(uy), _hptr(tot))
        if check:
            _check(st, "lbm_moments")
        return rho, ux, uy, tot

    def moments_device(self, rho=None, ux=None, uy=None, check=True):
        n = self.nx * self.ny
        tot = np.empty(3)
        st = self._L.lbm_moments_device(self._h, _dptr(rho, n), _dptr(ux, n), _dptr(uy, n), _hptr(tot))
        if check:
            _check(st, "lbm_moments_device")
        return tot

    def totals(self, check=True):
        return self.moments(fields=False, check=check)[3]

    # support calls -----------------------------------------------------------
    def get_f(self):
        f = np.empty((9, self.ny, self.nx))
        _check(self._L.lbm_get_f(self._h, _hptr(f)), "lbm_get_f")
        return f

    def sample_f(self, xs, ys):
        """f_i at the listed sites, shape (n, 9)."""
        xs = np.ascontiguousarray(xs, dtype=np.int32)
        ys = np.ascontiguousarray(ys, dtype=np.int32)
        assert xs.shape == ys.shape and xs.ndim == 1
        out = np.empty((len(xs), 9))
        _check(self._L.lbm_sample_f(self._h, len(xs), _hptr(xs), _hptr(ys), _hptr(out)), "lbm_sample_f")
        return out

    def set_f(self, f):
        f = _host(f, (9, self.ny, self.nx))
        _check(self._L.lbm_set_f(self._h, _hptr(f)), "lbm_set_f")
        return self

    def set_stream(self, stream):
        """Launch on a torch.cuda.Stream (its raw handle; 0 is the null
        stream), or on the library's own stream when `stream` is None."""
        if stream is None:
            _check(self._L.lbm_use_own_stream(self._h), "lbm_use_own_stream")
        else:
            _check(self._L.lbm_set_stream(self._h, ctypes.c_void_p(stream.cuda_stream)), "lbm_set_stream")
        self._stream_ref = stream
        return self

    @property
    def stream_handle(self):
        return self._L.lbm_get_stream(self._h) or 0

    def set_tile(self, vx, nw, h, flags=None):
        """Kernel shape (see lbm_set_tile); flags default to the current ones."""
        if flags is None:
            flags = self.get_tile()[3]
        _check(self._L.lbm_set_tile(self._h, int(vx), int(nw), int(h), int(flags)), "lbm_set_tile")
        return self

    def autotune(self, reps=5, use_cache=True):
        """Time the candidate kernel shapes on this lattice and keep the fastest."""
        _check(self._L.lbm_autotune(self._h, int(reps), int(bool(use_cache))), "lbm_autotune")
        return self.get_tile()

    def get_tile(self):
        v, w, h, f = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(self._L.lbm_get_tile(self._h, ctypes.byref(v), ctypes.byref(w), ctypes.byref(h), ctypes.byref(f)),
               "lbm_get_tile")
        return v.value, w.value, h.value, f.value

    @property
    def time(self):
        return self._L.lbm_time(self._h)

    @property
    def footprint(self):
        return footprint_bytes(self.nx, self.ny, self.dtype)
