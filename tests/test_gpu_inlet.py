"""GPU parity of the Fig. 1 boundaries (oscillating-density inlet at x = 0,
rho = 1 at the far end; Sec. 4) against the FP64 oracle, through the C ABI:
FP64 1e-12 and FP32 1e-5 max relative error in f, the shifted forms within
their tile-test bounds, every tile shape bitwise the same."""
import numpy as np
import pytest

import oracle
from gpu_util import max_rel_err, smooth_random_state

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_0707_2437_amd as lbm  # noqa: E402

TOL = {"f64": 1e-12, "f32": 1e-5, "f32s": 1e-5, "f16s": 2e-3}
DTYPES = ["f64", "f32", "f32s", "f16s"]
TILES = [(1, 8, 0, 18), (2, 8, 0, 18), (4, 8, 0, 16), (2, 16, 0, 18), (1, 1, 1, 0), (2, 4, 8, 15)]


def run_gpu(nx, ny, tau, c2, dtype, steps, fields, amp, period, tile=None, model=lbm.MODEL_FORCING):
    with lbm.Lattice(nx, ny, tau, c2, dtype, model=model) as L:
        if tile:
            L.set_tile(*tile)
        L.set_x_boundaries(lbm.XBC_INLET_OUTLET, amp, period)
        L.init(*fields)
        L.step(steps)
        return L.get_f()


def run_ref(nx, ny, tau, c2, steps, fields, amp, period, model=oracle.MODEL_FORCING):
    o = oracle.Oracle(nx, ny, tau, c2, model=model).set_x_boundaries(oracle.XBC_INLET_OUTLET, amp, period)
    return o.init(*fields).step(steps).get_f()


@pytest.mark.parametrize("c2", [0.09, 0.64])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_fig1_setup_parity(c2, dtype):
    """A 600 x 4 channel driven for 1500 steps (the wave reaches the outlet
    and is reflected for c^2 = 0.64)."""
    fields = (None, None, None)
    f = run_gpu(600, 4, 0.6, c2, dtype, 1500, fields, 0.01, 250.0)
    err = max_rel_err(f, run_ref(600, 4, 0.6, c2, 1500, fields, 0.01, 250.0))
    print(f"Fig. 1 set-up c2={c2} {dtype}: max rel err f = {err:.3e}")
    assert err <= TOL[dtype]


@pytest.mark.parametrize("dtype", DTYPES)
def test_boundaries_shapes_and_tiles(dtype):
    """Ragged shapes, a non-trivial interior state, every tile shape bitwise
    the same, and the oracle."""
    for nx, ny in [(397, 131), (5, 7), (130, 9), (258, 4)]:
        fields = smooth_random_state(nx, ny, seed=3 * nx + ny)
        outs = [run_gpu(nx, ny, 0.7, 0.3, dtype, 40, fields, 0.05, 17.0, tile=t) for t in TILES]
        for t, o in zip(TILES[1:], outs[1:]):
            assert np.array_equal(o, outs[0]), (nx, ny, t)
        err = max_rel_err(outs[0], run_ref(nx, ny, 0.7, 0.3, 40, fields, 0.05, 17.0))
        assert err <= TOL[dtype], (nx, ny, err)


def test_boundaries_with_equilibrium_model():
    fields = smooth_random_state(130, 9, seed=5)
    f = run_gpu(130, 9, 0.7, 0.45, "f64", 60, fields, 0.05, 17.0, model=lbm.MODEL_EQUILIBRIUM)
    fr = run_ref(130, 9, 0.7, 0.45, 60, fields, 0.05, 17.0, model=oracle.MODEL_EQUILIBRIUM)
    assert max_rel_err(f, fr) <= TOL["f64"]


def test_boundaries_switch_off_and_rules():
    nx, ny = 64, 6
    fields = smooth_random_state(nx, ny, seed=8)
    o = oracle.Oracle(nx, ny, 0.7, 0.3).set_x_boundaries(oracle.XBC_INLET_OUTLET, 0.05, 17.0).init(*fields)
    with lbm.Lattice(nx, ny, 0.7, 0.3, "f64") as L:
        L.set_x_boundaries(lbm.XBC_INLET_OUTLET, 0.05, 17.0).init(*fields).step(20)
        o.step(20)
        L.set_x_boundaries(lbm.XBC_PERIODIC).step(20)
        o.set_x_boundaries(oracle.XBC_PERIODIC).step(20)
        assert max_rel_err(L.get_f(), o.get_f()) <= TOL["f64"]
        for args in [(1, 1.0, 10.0), (1, 0.1, 0.0), (1, 0.1, float("nan")), (7, 0.1, 10.0)]:
            with pytest.raises(lbm.LBMError) as ei:
                L.set_x_boundaries(*args)
            assert ei.value.status == lbm.EINVAL
    with lbm.Lattice(4, 4, 0.7, 0.3, "f64") as L:
        with pytest.raises(lbm.LBMError):
            L.set_x_boundaries(lbm.XBC_INLET_OUTLET, 0.1, 10.0)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_fig1_sound_speed_over_alpha(dtype):
    """Fig. 1 on the GPU: the Fig. 1 set-up (inlet period 500 steps, 2400 x 4
    channel, tau = 0.6) for alpha from -0.8 to 0.3 (c_e = 0.18 ... 1.06); the
    phase speed between probes at x = 200 and 400 in the periodic regime, and
    u / delta rho there, against c_e = sqrt(1/3 - alpha) (Eq. 8). The window
    closes before the outlet's echo reaches the probes."""
    nx, ny, tau, T, amp, x1, x2 = 2400, 4, 0.6, 500, 1e-3, 200, 400
    w = 2 * np.pi / T
    rows = []
    for alpha in (-0.8, -0.6, -0.3, 0.0, 0.2, 0.3):
        c2 = 1.0 / 3.0 - alpha
        c = np.sqrt(c2)
        t0 = int(x2 / c + 3 * T)
        t1 = t0 + 4 * T
        assert (2 * nx - x2) / c > t1
        R, U = np.empty((t1 - t0, 2)), np.empty((t1 - t0, 2))
        with lbm.Lattice(nx, ny, tau, c2, dtype) as L:
            L.set_x_boundaries(lbm.XBC_INLET_OUTLET, amp, T).init()
            L.step(t0)
            for t in range(t0, t1):
                rho, ux, _, _ = L.moments()
                R[t - t0], U[t - t0] = rho[0, [x1, x2]] - 1, ux[0, [x1, x2]]
                L.step(1)
        ph = np.exp(-1j * w * np.arange(t0, t1))[:, None]
        a, b = (R * ph).mean(0), (U * ph).mean(0)
        dphi = np.angle(a[0] / a[1])
        dphi += 2 * np.pi * np.round((w / c * (x2 - x1) - dphi) / (2 * np.pi))
        speed = w * (x2 - x1) / dphi
        ratio = abs(b[1] / a[1])
        rows.append((alpha, c, speed, ratio))
        print(f"Fig. 1 {dtype}: alpha = {alpha:+.2f}  c_e = {c:.4f}  measured {speed:.4f}  u/drho {ratio:.4f}")
    for alpha, c, speed, ratio in rows:
        assert abs(speed / c - 1) < 1e-2, alpha
        assert abs(ratio / c - 1) < 2e-2, alpha
