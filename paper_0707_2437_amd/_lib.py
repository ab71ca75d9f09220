"""ctypes loader for liblbm.so (argument marshalling only).

The shared library is the product: every step of the method runs in its HIP
kernels. There is no fallback: if the library is missing or cannot be loaded,
the first use raises LibraryNotBuilt.
"""
import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "liblbm.so")

_lib = None


class LibraryNotBuilt(RuntimeError):
    pass


_dp = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p
_i = ctypes.c_int
_d = ctypes.c_double

# name: (restype, argtypes) -- mirrors include/liblbm.h
SIGNATURES = {
    "lbm_create": (_vp, [_i, _i, _d, _d, _i]),
    "lbm_last_error": (_i, []),
    "lbm_strerror": (ctypes.c_char_p, [_i]),
    "lbm_destroy": (None, [_vp]),
    "lbm_init": (_i, [_vp, _vp, _vp, _vp]),
    "lbm_set_model": (_i, [_vp, _i]),
    "lbm_set_x_boundaries": (_i, [_vp, _i, _d, _d]),
    "lbm_set_c2_field": (_i, [_vp, _vp]),
    "lbm_set_c2_field_device": (_i, [_vp, _vp]),
    "lbm_init_device": (_i, [_vp, _vp, _vp, _vp]),
    "lbm_step": (_i, [_vp, _i]),
    "lbm_moments": (_i, [_vp, _vp, _vp, _vp, _vp]),
    "lbm_moments_device": (_i, [_vp, _vp, _vp, _vp, _vp]),
    "lbm_get_f": (_i, [_vp, _vp]),
    "lbm_set_f": (_i, [_vp, _vp]),
    "lbm_sample_f": (_i, [_vp, _i, _vp, _vp, _vp]),
    "lbm_set_stream": (_i, [_vp, _vp]),
    "lbm_use_own_stream": (_i, [_vp]),
    "lbm_get_stream": (_vp, [_vp]),
    "lbm_time": (ctypes.c_longlong, [_vp]),
    "lbm_footprint_bytes": (ctypes.c_size_t, [_i, _i, _i]),
    "lbm_pool_create": (_vp, [ctypes.c_size_t, _i]),
    "lbm_pool_last_error": (_i, []),
    "lbm_pool_destroy": (None, [_vp]),
    "lbm_pool_slot_bytes": (ctypes.c_size_t, [_i, _i, _i]),
    "lbm_pool_used_bytes": (ctypes.c_size_t, [_vp]),
    "lbm_pool_budget_bytes": (ctypes.c_size_t, [_vp]),
    "lbm_pool_device_bytes": (ctypes.c_size_t, [_vp]),
    "lbm_pool_add": (_i, [_vp, _i, _i, _d, _d]),
    "lbm_pool_remove": (_i, [_vp, _i]),
    "lbm_pool_init": (_i, [_vp, _i, _vp, _vp, _vp]),
    "lbm_pool_init_device": (_i, [_vp, _i, _vp, _vp, _vp]),
    "lbm_pool_step": (_i, [_vp, _vp, _vp, _i]),
    "lbm_pool_step_noalloc": (_i, [_vp, _vp, _vp, _i]),
    "lbm_pool_sync": (_i, [_vp]),
    "lbm_pool_persistent_members": (_i, [_vp]),
    "lbm_pool_moments": (_i, [_vp, _i, _vp, _vp, _vp, _vp]),
    "lbm_pool_totals_device": (_i, [_vp, _i, _vp]),
    "lbm_pool_get_f": (_i, [_vp, _i, _vp]),
    "lbm_pool_time": (ctypes.c_longlong, [_vp, _i]),
    "lbm_pool_set_mode": (_i, [_vp, _i, _i]),
    "lbm_pool_set_tile": (_i, [_vp, _i, _i, _i]),
    "lbm_pool_get_tile": (_i, [_vp, _vp, _vp, _vp]),
    "lbm_pool_set_items": (_i, [_vp, _i]),
    "lbm_pool_set_stream": (_i, [_vp, _vp]),
    "lbm_set_tile": (_i, [_vp, _i, _i, _i, _i]),
    "lbm_autotune": (_i, [_vp, _i, _i]),
    "lbm_pool_autotune": (_i, [_vp, _vp, _i, _i, _i]),
    "lbm_get_tile": (_i, [_vp, _vp, _vp, _vp, _vp]),
}


def lib():
    """The loaded liblbm.so (loaded once)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise LibraryNotBuilt(f"{LIB_PATH} is missing: build it with `python -m paper_0707_2437_amd.build`")
    try:
        L = ctypes.CDLL(LIB_PATH, mode=ctypes.RTLD_LOCAL)
    except OSError as e:
        raise LibraryNotBuilt(f"cannot load {LIB_PATH}: {e}") from e
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L
