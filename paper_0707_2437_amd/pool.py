"""Python binding of the lbm_pool C ABI (batched and served forms)."""
import ctypes
import sys

import numpy as np

from ._lib import lib
from .lattice import LBMError, _check, _dptr, _dtype_code, _host, _hptr

GROUPED, GRAPH, PERSISTENT = 0, 1, 2


class Pool:
    """Resident lattices of one dtype under a device-memory budget, stepped
    together by batched launches."""

    def __init__(self, budget_bytes, dtype="f32"):
        self._L = lib()
        self.dtype = _dtype_code(dtype)
        h = self._L.lbm_pool_create(int(budget_bytes), self.dtype)
        if not h:
            raise LBMError(self._L.lbm_pool_last_error(), "lbm_pool_create")
        self._h = ctypes.c_void_p(h)
        self.shapes = {}
        self._stream_ref = None

    def close(self):
        if getattr(self, "_h", None):
            self._L.lbm_pool_destroy(self._h)
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

    @staticmethod
    def slot_bytes(nx, ny, dtype):
        return lib().lbm_pool_slot_bytes(int(nx), int(ny), _dtype_code(dtype))

    @property
    def used_bytes(self):
        return self._L.lbm_pool_used_bytes(self._h)

    @property
    def budget_bytes(self):
        return self._L.lbm_pool_budget_bytes(self._h)

    @property
    def device_bytes(self):
        """Device memory the pool holds for its slots (never above the budget)."""
        return self._L.lbm_pool_device_bytes(self._h)

    def add(self, nx, ny, tau, c2):
        s = self._L.lbm_pool_add(self._h, int(nx), int(ny), float(tau), float(c2))
        if s < 0:
            raise LBMError(s, "lbm_pool_add")
        self.shapes[s] = (int(ny), int(nx))
        return s

    def try_add(self, nx, ny, tau, c2):
        """Slot id, or None when the budget (or device memory) is exhausted."""
        s = self._L.lbm_pool_add(self._h, int(nx), int(ny), float(tau), float(c2))
        if s == -2:
            return None
        if s < 0:
            raise LBMError(s, "lbm_pool_add")
        self.shapes[s] = (int(ny), int(nx))
        return s

    def remove(self, slot):
        _check(self._L.lbm_pool_remove(self._h, int(slot)), "lbm_pool_remove")
        self.shapes.pop(slot, None)

    def init(self, slot, rho=None, ux=None, uy=None):
        shape = self.shapes[slot]
        rho, ux, uy = _host(rho, shape), _host(ux, shape), _host(uy, shape)
        _check(self._L.lbm_pool_init(self._h, int(slot), _hptr(rho), _hptr(ux), _hptr(uy)), "lbm_pool_init")

    def init_device(self, slot, rho=None, ux=None, uy=None):
        n = self.shapes[slot][0] * self.shapes[slot][1]
        _check(self._L.lbm_pool_init_device(self._h, int(slot), _dptr(rho, n), _dptr(ux, n), _dptr(uy, n)),
               "lbm_pool_init_device")

    def step(self, slots, nsteps):
        slots = np.ascontiguousarray(slots, dtype=np.int32)
        if np.isscalar(nsteps):
            nsteps = np.full(len(slots), int(nsteps), dtype=np.int32)
        nsteps = np.ascontiguousarray(nsteps, dtype=np.int32)
        assert slots.shape == nsteps.shape
        _check(self._L.lbm_pool_step(self._h, _hptr(slots), _hptr(nsteps), len(slots)), "lbm_pool_step")

    def step_noalloc(self, slots, nsteps):
        """lbm_pool_step_noalloc: as step, with no device allocation in the call."""
        slots = np.ascontiguousarray(slots, dtype=np.int32)
        if np.isscalar(nsteps):
            nsteps = np.full(len(slots), int(nsteps), dtype=np.int32)
        nsteps = np.ascontiguousarray(nsteps, dtype=np.int32)
        assert slots.shape == nsteps.shape
        _check(self._L.lbm_pool_step_noalloc(self._h, _hptr(slots), _hptr(nsteps), len(slots)),
               "lbm_pool_step_noalloc")

    def sync(self):
        _check(self._L.lbm_pool_sync(self._h), "lbm_pool_sync")

    def persistent_members(self):
        """Workgroups that took part in the last persistent launch."""
        n = self._L.lbm_pool_persistent_members(self._h)
        if n < 0:
            raise LBMError(n, "lbm_pool_persistent_members")
        return n

    def moments(self, slot, fields=True, check=True):
        shape = self.shapes[slot]
        rho = np.empty(shape) if fields else None
        ux = np.empty(shape) if fields else None
        uy = np.empty(shape) if fields else None
        tot = np.empty(3)
        st = self._L.lbm_pool_moments(self._h, int(slot), _hptr(rho), _hptr(ux), _hptr(uy), _hptr(tot))
        if check:
            _check(st, "lbm_pool_moments")
        return rho, ux, uy, tot, st

    def totals(self, slot):
        """(totals, status); status is ENONFINITE for a blown-up lattice."""
        _, _, _, tot, st = self.moments(slot, fields=False, check=False)
        if st not in (0, -5):
            raise LBMError(st, "lbm_pool_moments")
        return tot, st

    def totals_device(self, slot, out):
        """lbm_pool_totals_device: the slot's totals into `out`, a float64 CUDA
        tensor of 3 elements (or a view of 3), asynchronously on the pool's stream."""
        _check(self._L.lbm_pool_totals_device(self._h, int(slot), _dptr(out, 3)), "lbm_pool_totals_device")

    def get_f(self, slot):
        ny, nx = self.shapes[slot]
        f = np.empty((9, ny, nx))
        _check(self._L.lbm_pool_get_f(self._h, int(slot), _hptr(f)), "lbm_pool_get_f")
        return f

    def time(self, slot):
        return self._L.lbm_pool_time(self._h, int(slot))

    def set_mode(self, mode, max_grid=0):
        _check(self._L.lbm_pool_set_mode(self._h, int(mode), int(max_grid)), "lbm_pool_set_mode")

    def set_tile(self, vx, nw, flags=0):
        _check(self._L.lbm_pool_set_tile(self._h, int(vx), int(nw), int(flags)), "lbm_pool_set_tile")

    def autotune(self, slots, reps=3, use_cache=True):
        """Time the batched kernels' tile shapes on one launch over `slots` and keep the fastest."""
        slots = np.ascontiguousarray(slots, dtype=np.int32)
        _check(self._L.lbm_pool_autotune(self._h, _hptr(slots), len(slots), int(reps), int(bool(use_cache))),
               "lbm_pool_autotune")
        return self.get_tile()

    def set_items(self, tiles_per_item):
        _check(self._L.lbm_pool_set_items(self._h, int(tiles_per_item)), "lbm_pool_set_items")

    def get_tile(self):
        v, w, f = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(self._L.lbm_pool_get_tile(self._h, ctypes.byref(v), ctypes.byref(w), ctypes.byref(f)),
               "lbm_pool_get_tile")
        return v.value, w.value, f.value

    def set_stream(self, stream):
        ptr = None if stream is None else ctypes.c_void_p(stream.cuda_stream)
        _check(self._L.lbm_pool_set_stream(self._h, ptr), "lbm_pool_set_stream")
        self._stream_ref = stream
