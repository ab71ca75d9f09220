"""ctypes wrapper around liblbmref.so, the FP64 C oracle (TEST INFRASTRUCTURE).

Mirrors the C interface in lbmref.h one call to one method; no arithmetic of
the method lives here. Fields are numpy float64 arrays of shape (ny, nx);
populations have shape (9, ny, nx).
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_LIB = os.path.join(_HERE, "liblbmref.so")

_libs = {}

_dp = ctypes.POINTER(ctypes.c_double)


def _ptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(_dp)


def load(path=None):
    """Load (once) the oracle library at `path` (default: $LBMREF_LIB, else the
    in-tree build; the variable lets the mutation tests swap in a planted-bug
    build of the same source)."""
    path = os.path.abspath(path or os.environ.get("LBMREF_LIB") or DEFAULT_LIB)
    if path in _libs:
        return _libs[path]
    if not os.path.exists(path):
        raise RuntimeError(f"oracle library {path} is not built; run `make -C oracle`")
    lib = ctypes.CDLL(path, mode=ctypes.RTLD_LOCAL)
    lib.lbmref_lattice.argtypes = [ctypes.POINTER(ctypes.c_int), _dp]
    lib.lbmref_lattice.restype = None
    lib.lbmref_alpha.argtypes = [ctypes.c_double]
    lib.lbmref_alpha.restype = ctypes.c_double
    lib.lbmref_equilibrium.argtypes = [ctypes.c_double] * 3 + [_dp]
    lib.lbmref_equilibrium.restype = None
    lib.lbmref_source.argtypes = [ctypes.c_double] * 3 + [_dp]
    lib.lbmref_equilibrium_c2.argtypes = [ctypes.c_double] * 4 + [_dp]
    lib.lbmref_equilibrium_c2.restype = None
    lib.lbmref_set_model.argtypes = [ctypes.c_void_p, ctypes.c_int]
    lib.lbmref_set_model.restype = ctypes.c_int
    lib.lbmref_source.restype = None
    lib.lbmref_set_x_boundaries.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_double]
    lib.lbmref_set_x_boundaries.restype = ctypes.c_int
    lib.lbmref_set_c2_field.argtypes = [ctypes.c_void_p, _dp]
    lib.lbmref_set_c2_field.restype = ctypes.c_int
    lib.lbmref_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double]
    lib.lbmref_create.restype = ctypes.c_void_p
    lib.lbmref_last_error.argtypes = []
    lib.lbmref_last_error.restype = ctypes.c_int
    lib.lbmref_destroy.argtypes = [ctypes.c_void_p]
    lib.lbmref_destroy.restype = None
    lib.lbmref_init.argtypes = [ctypes.c_void_p, _dp, _dp, _dp]
    lib.lbmref_init.restype = ctypes.c_int
    lib.lbmref_step.argtypes = [ctypes.c_void_p, ctypes.c_int]
    lib.lbmref_step.restype = ctypes.c_int
    lib.lbmref_moments.argtypes = [ctypes.c_void_p, _dp, _dp, _dp, _dp]
    lib.lbmref_moments.restype = ctypes.c_int
    lib.lbmref_get_f.argtypes = [ctypes.c_void_p, _dp]
    lib.lbmref_get_f.restype = ctypes.c_int
    lib.lbmref_set_f.argtypes = [ctypes.c_void_p, _dp]
    lib.lbmref_set_f.restype = ctypes.c_int
    lib.lbmref_time.argtypes = [ctypes.c_void_p]
    lib.lbmref_time.restype = ctypes.c_longlong
    lib.lbmref_set_threads.argtypes = [ctypes.c_int]
    lib.lbmref_set_threads.restype = None
    lib.lbmref_get_threads.argtypes = []
    lib.lbmref_get_threads.restype = ctypes.c_int
    _libs[path] = lib
    return lib


def lattice(lib=None):
    """(e, w): e int array (9, 2), w float64 array (9,), as the oracle evaluates them."""
    lib = lib or load()
    e = (ctypes.c_int * 18)()
    w = np.zeros(9)
    lib.lbmref_lattice(e, _ptr(w))
    return np.array(list(e), dtype=np.int64).reshape(9, 2), w


def alpha(c2, lib=None):
    return (lib or load()).lbmref_alpha(float(c2))


def equilibrium(rho, ux, uy, lib=None):
    out = np.zeros(9)
    (lib or load()).lbmref_equilibrium(float(rho), float(ux), float(uy), _ptr(out))
    return out


def equilibrium_c2(c2, rho, ux, uy, lib=None):
    """The altered equilibrium of the equilibrium model (lbmref.h)."""
    out = np.zeros(9)
    (lib or load()).lbmref_equilibrium_c2(float(c2), float(rho), float(ux), float(uy), _ptr(out))
    return out


MODEL_FORCING, MODEL_EQUILIBRIUM = 0, 1
XBC_PERIODIC, XBC_INLET_OUTLET = 0, 1


def source(alpha_, gx, gy, lib=None):
    out = np.zeros(9)
    (lib or load()).lbmref_source(float(alpha_), float(gx), float(gy), _ptr(out))
    return out


def set_threads(n, lib=None):
    (lib or load()).lbmref_set_threads(int(n))


def get_threads(lib=None):
    return (lib or load()).lbmref_get_threads()


class OracleError(RuntimeError):
    def __init__(self, status, what):
        super().__init__(f"{what}: oracle status {status}")
        self.status = status


class Oracle:
    """One periodic lattice stepped by the FP64 oracle."""

    def __init__(self, nx, ny, tau, c2, lib_path=None, model=MODEL_FORCING):
        self.lib = load(lib_path)
        self.nx, self.ny, self.tau, self.c2 = int(nx), int(ny), float(tau), float(c2)
        h = self.lib.lbmref_create(self.nx, self.ny, self.tau, self.c2)
        if not h:
            raise OracleError(self.lib.lbmref_last_error(), "lbmref_create")
        self._h = ctypes.c_void_p(h)
        if model != MODEL_FORCING:
            self._check(self.lib.lbmref_set_model(self._h, int(model)), "lbmref_set_model")

    def close(self):
        if getattr(self, "_h", None):
            self.lib.lbmref_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def _check(self, st, what):
        if st != 0:
            raise OracleError(st, what)

    def _field(self, a):
        if a is None:
            return None
        a = np.ascontiguousarray(a, dtype=np.float64)
        if a.shape != (self.ny, self.nx):
            a = np.ascontiguousarray(np.broadcast_to(a, (self.ny, self.nx)))
        return a

    def set_x_boundaries(self, mode, amplitude=0.0, period=0.0):
        """XBC_PERIODIC, or XBC_INLET_OUTLET (Fig. 1: rho_in(t) at x = 0, rho = 1 at x = nx - 1)."""
        self._check(self.lib.lbmref_set_x_boundaries(self._h, int(mode), float(amplitude), float(period)),
                    "set_x_boundaries")
        return self

    def set_c2_field(self, c2):
        """Per-site c_e^2 (shape (ny, nx), broadcast if smaller); None: uniform again."""
        c2 = self._field(c2)
        self._check(self.lib.lbmref_set_c2_field(self._h, _ptr(c2)), "set_c2_field")
        return self

    def init(self, rho=None, ux=None, uy=None):
        rho, ux, uy = self._field(rho), self._field(ux), self._field(uy)
        self._check(self.lib.lbmref_init(self._h, _ptr(rho), _ptr(ux), _ptr(uy)), "init")
        return self

    def step(self, n=1):
        self._check(self.lib.lbmref_step(self._h, int(n)), "step")
        return self

    def moments(self, check=True):
        """(rho, ux, uy, totals) of the current state; totals = (M, Px, Py)."""
        rho = np.empty((self.ny, self.nx))
        ux = np.empty_like(rho)
        uy = np.empty_like(rho)
        tot = np.empty(3)
        st = self.lib.lbmref_moments(self._h, _ptr(rho), _ptr(ux), _ptr(uy), _ptr(tot))
        if check:
            self._check(st, "moments")
        return rho, ux, uy, tot

    def get_f(self):
        f = np.empty((9, self.ny, self.nx))
        self._check(self.lib.lbmref_get_f(self._h, _ptr(f)), "get_f")
        return f

    def set_f(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64)
        assert f.shape == (9, self.ny, self.nx)
        self._check(self.lib.lbmref_set_f(self._h, _ptr(f)), "set_f")
        return self

    @property
    def time(self):
        return self.lib.lbmref_time(self._h)
