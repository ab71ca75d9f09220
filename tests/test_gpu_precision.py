"""Precision forms at the precision workload's full size: a periodic
8192 x 8192 shear wave u_x = 0.01 sin(2 pi y / 8192), tau = 0.7, c^2 = 0.25,
5000 steps, shifted storage g_i = f_i - w_i in FP32 and in FP16 with FP32
arithmetic, against the FP64 oracle. The state is x-invariant, so the oracle
runs on an 8192 (y) x 4 (x) strip, which is bitwise the full-width result;
the GPU run must keep every sampled column bitwise identical. Errors are
reported per result: max relative error in f, and the errors of rho - 1 and
u_x relative to the wave amplitude."""
import numpy as np
import pytest

import oracle
from gpu_util import max_rel_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_0707_2437_amd as lbm  # noqa: E402
from paper_0707_2437_amd import workloads  # noqa: E402

N, TAU, C2, STEPS, AMP = 8192, 0.7, 0.25, 5000, 0.01
# FP32: the FP32 bar of the plain form (1e-5 in f). The state barely changes
# over the run (shear decay exp(-nu k^2 t) = exp(-2e-4)), so the same FP32
# roundings of the momentum-carrying terms recur every step and add up
# linearly: measured 5.9e-6 in f and 2.0e-4 of the amplitude in u.
# FP16 keeps ~11 bits of g = f - w: measured 4.0e-5 in f and 6.5e-4 of the
# amplitude in u; bounds 5x above.
BOUNDS = {"f32s": {"f": 1e-5, "u": 1e-3}, "f16s": {"f": 2e-4, "u": 5e-3}}


@pytest.fixture(scope="module")
def oracle_strip():
    _, ux, _ = workloads.shear_wave_fields(4, N, amp=AMP)
    o = oracle.Oracle(4, N, TAU, C2).init(None, ux, None).step(STEPS)
    f = o.get_f()
    rho, uxo, _, _ = o.moments()
    assert np.all(f == f[:, :, :1])  # x-invariant, bitwise
    return f[:, :, 0], rho[:, 0], uxo[:, 0]


@pytest.mark.parametrize("dtype", ["f32s", "f16s"])
def test_shear_wave_precision_full_size(dtype, oracle_strip):
    fref, rref, uref = oracle_strip
    _, ux, _ = workloads.shear_wave_fields(N, N, amp=AMP)
    ys = np.arange(0, N, 7)
    with lbm.Lattice(N, N, TAU, C2, dtype) as L:
        L.init(None, ux, None).step(STEPS)
        cols = {}
        for x in (0, 1, 4095, 4096, N - 1):
            cols[x] = L.sample_f(np.full(len(ys), x), ys)  # (n, 9)
        rho, uxg, _, tot = L.moments()
    for x in cols:
        assert np.array_equal(cols[x], cols[0]), x  # every column identical
    f_gpu = cols[0].T  # (9, n)
    err_f = max_rel_err(f_gpu, fref[:, ys])
    err_rho = np.max(np.abs(rho[:, 0] - rref)) / AMP
    err_u = np.max(np.abs(uxg[:, 0] - uref)) / AMP
    print(f"{dtype}: max rel err f {err_f:.3e}; |rho - rho_ref| / amp {err_rho:.3e}; "
          f"|u - u_ref| / amp {err_u:.3e}")
    assert err_f <= BOUNDS[dtype]["f"]
    assert err_u <= BOUNDS[dtype]["u"]
    assert np.all(rho == rho[:, :1])
