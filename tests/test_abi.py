"""Host-side checks of the C ABI that need no GPU: the built library and the
oracle export every function their headers declare, the Python binding
mirrors the header, and argument validation rejects what Sec. 2-4 rule out
before any device work."""
import ctypes
import os
import re

import pytest

import paper_0707_2437_amd as lbm
from paper_0707_2437_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions(header):
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm(?:ref)?_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    names = declared_functions(os.path.join(ROOT, "include", "liblbm.h"))
    assert "lbm_create" in names and "lbm_step" in names
    L = ctypes.CDLL(_lib.LIB_PATH, mode=ctypes.RTLD_LOCAL)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_binding_mirrors_header():
    names = declared_functions(os.path.join(ROOT, "include", "liblbm.h"))
    assert sorted(_lib.SIGNATURES) == names


def test_oracle_exports_every_declared_symbol():
    names = declared_functions(os.path.join(ROOT, "oracle", "lbmref.h"))
    L = ctypes.CDLL(os.path.join(ROOT, "oracle", "liblbmref.so"), mode=ctypes.RTLD_LOCAL)
    assert not [n for n in names if not hasattr(L, n)]


@pytest.mark.parametrize("args", [(2, 8, 0.8, 0.2, 0), (8, 2, 0.8, 0.2, 0), (8, 8, 0.5, 0.2, 0),
                                  (8, 8, 0.4, 0.2, 1), (8, 8, float("nan"), 0.2, 0), (8, 8, float("inf"), 0.2, 0),
                                  (8, 8, 0.8, 0.0, 0), (8, 8, 0.8, -1.0, 2), (8, 8, 0.8, float("nan"), 3),
                                  (8, 8, 0.8, 0.2, 4), (8, 8, 0.8, 0.2, -1),
                                  # one row past the largest lattice whose planes fit 32-bit byte offsets
                                  (32768, 32704, 0.8, 0.2, 1), (32768, 16368, 0.8, 0.2, 0)])
def test_create_rejects_invalid_arguments_before_device_work(args):
    L = _lib.lib()
    assert not L.lbm_create(*args)
    assert L.lbm_last_error() == lbm.EINVAL


def test_largest_lattices_accepted():
    """The largest lattices the maximum-size GPU tests create (32768 wide)."""
    L = _lib.lib()
    assert L.lbm_footprint_bytes(32768, 32703, 1) > 0 and L.lbm_footprint_bytes(32768, 32704, 1) == 0
    assert L.lbm_footprint_bytes(32768, 16367, 0) > 0 and L.lbm_footprint_bytes(32768, 16368, 0) == 0


def test_footprint_bytes():
    L = _lib.lib()
    assert L.lbm_footprint_bytes(2, 8, 0) == 0
    assert L.lbm_footprint_bytes(8, 8, 7) == 0
    f32 = L.lbm_footprint_bytes(4096, 4096, 1)
    f64 = L.lbm_footprint_bytes(4096, 4096, 0)
    f16 = L.lbm_footprint_bytes(4096, 4096, 3)
    # A + B: 18 planes of 4096 x (4096 + padding) entries
    assert 18 * 4096 * 4096 * 4 <= f32 <= 1.05 * 18 * 4096 * 4096 * 4
    assert 1.9 * f32 <= f64 <= 2.1 * f32
    assert 0.45 * f32 <= f16 <= 0.55 * f32


def test_null_handle_calls_are_errors():
    L = _lib.lib()
    assert L.lbm_step(None, 1) == lbm.EINVAL
    assert L.lbm_init(None, None, None, None) == lbm.EINVAL
    assert L.lbm_set_model(None, lbm.MODEL_EQUILIBRIUM) == lbm.EINVAL
    assert L.lbm_set_c2_field(None, None) == lbm.EINVAL
    assert L.lbm_set_x_boundaries(None, 0, 0.0, 0.0) == lbm.EINVAL
    assert L.lbm_set_c2_field_device(None, None) == lbm.EINVAL
    assert L.lbm_moments(None, None, None, None, None) == lbm.EINVAL
    assert L.lbm_time(None) == -1
    L.lbm_destroy(None)
    assert L.lbm_strerror(lbm.ENONFINITE) == b"non-finite conservation total"
