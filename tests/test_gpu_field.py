"""GPU parity of the c2 field (a speed of sound varying in space, Sec. 5
outlook) against the FP64 oracle, through the C ABI. Same bars as the
uniform lattice: FP64 1e-12 and FP32 1e-5 max relative error in f; the
shifted forms within their tile-test bounds; a uniform field gives the bits
of the uniform lattice; every vertical-stack shape gives the same bits."""
import numpy as np
import pytest

import oracle
from gpu_util import c1_rho, max_rel_err, smooth_random_state
from paper_0707_2437_amd import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_0707_2437_amd as lbm  # noqa: E402

TOL = {"f64": 1e-12, "f32": 1e-5, "f32s": 1e-5, "f16s": 2e-3}
DTYPES = ["f64", "f32", "f32s", "f16s"]
VSTACK_TILES = [(1, 8, 0, 18), (2, 8, 0, 18), (4, 8, 0, 16), (2, 16, 0, 18), (1, 4, 0, 16), (4, 16, 0, 18)]


def field(nx, ny, seed, c2=0.35, noise=0.05):
    return workloads.lens_c2_field(nx, ny, c2, depth=0.6, noise=noise, seed=seed)


def run_gpu(nx, ny, tau, c2, dtype, steps, fields, c2f, tile=None, device=False):
    with lbm.Lattice(nx, ny, tau, c2, dtype) as L:
        if tile:
            L.set_tile(*tile)
        if device:
            L.set_c2_field_device(torch.from_numpy(np.ascontiguousarray(c2f).ravel()).cuda())
        else:
            L.set_c2_field(c2f)
        L.init(*fields)
        L.step(steps)
        return L.get_f()


def run_ref(nx, ny, tau, c2, steps, fields, c2f):
    return oracle.Oracle(nx, ny, tau, c2).set_c2_field(c2f).init(*fields).step(steps).get_f()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_field_c1_parity_1000_steps(dtype):
    fields = (c1_rho(), None, None)
    c2f = field(64, 64, 1)
    f = run_gpu(64, 64, 0.8, 0.2, dtype, 1000, fields, c2f)
    err = max_rel_err(f, run_ref(64, 64, 0.8, 0.2, 1000, fields, c2f))
    print(f"field C1 {dtype}: max rel err f = {err:.3e}")
    assert err <= TOL[dtype]


@pytest.mark.parametrize("dtype", DTYPES)
def test_field_shapes_and_tiles(dtype):
    """Ragged shapes (strips, row groups and a tail), every vertical-stack
    shape bitwise the same, host and device field calls the same, and the oracle."""
    for nx, ny in [(397, 131), (5, 7), (130, 9), (258, 33)]:
        fields = smooth_random_state(nx, ny, seed=nx + 5 * ny)
        c2f = field(nx, ny, nx * ny)
        outs = [run_gpu(nx, ny, 0.7, 0.3, dtype, 30, fields, c2f, tile=t) for t in VSTACK_TILES]
        for t, o in zip(VSTACK_TILES[1:], outs[1:]):
            assert np.array_equal(o, outs[0]), (nx, ny, t)
        assert np.array_equal(run_gpu(nx, ny, 0.7, 0.3, dtype, 30, fields, c2f, device=True), outs[0]), (nx, ny)
        err = max_rel_err(outs[0], run_ref(nx, ny, 0.7, 0.3, 30, fields, c2f))
        assert err <= TOL[dtype], (nx, ny, err)


@pytest.mark.parametrize("dtype", DTYPES)
def test_uniform_field_is_the_uniform_lattice_bitwise(dtype):
    nx, ny = 300, 41
    fields = smooth_random_state(nx, ny, seed=11)
    with lbm.Lattice(nx, ny, 0.7, 0.45, dtype) as L:
        f0 = L.init(*fields).step(25).get_f()
    f1 = run_gpu(nx, ny, 0.7, 0.9, dtype, 25, fields, np.full((ny, nx), 0.45))
    assert np.array_equal(f0, f1)


def test_field_changed_between_steps():
    """alpha varying in time: two fields alternated every 5 steps."""
    nx, ny = 130, 40
    fields = smooth_random_state(nx, ny, seed=3)
    fa, fb = field(nx, ny, 1), field(nx, ny, 2, c2=0.5)
    o = oracle.Oracle(nx, ny, 0.75, 0.3).init(*fields)
    with lbm.Lattice(nx, ny, 0.75, 0.3, "f64") as L:
        L.init(*fields)
        for k in range(6):
            c = fa if k % 2 == 0 else fb
            L.set_c2_field(c).step(5)
            o.set_c2_field(c).step(5)
        # and back to the uniform c2
        L.set_c2_field(None).step(5)
        o.set_c2_field(None).step(5)
        assert max_rel_err(L.get_f(), o.get_f()) <= TOL["f64"]


def test_interface_reflection_matches_oracle():
    """The oracle's interface test case (a pulse meeting a jump in c) on the GPU."""
    nx, ny, x0, xi, sigma, tau, eps, cA2, cB2 = 1400, 3, 500, 800, 12.0, 0.55, 1e-4, 0.25, 0.64
    x = np.arange(nx)[None, :] * np.ones((ny, 1))
    g = np.exp(-0.5 * ((x - x0) / sigma) ** 2)
    c2f = np.where(x < xi, cA2, cB2)
    fields = (1 + eps * g, 0.5 * eps * g, None)
    f = run_gpu(nx, ny, tau, cA2, "f64", 900, fields, c2f)
    assert max_rel_err(f, run_ref(nx, ny, tau, cA2, 900, fields, c2f)) <= TOL["f64"]


def test_field_rules():
    with lbm.Lattice(16, 12, 0.7, 0.3, "f32") as L:
        L.set_tile(1, 1, 4, 0)  # a march-form shape
        L.set_c2_field(np.full((12, 16), 0.3))
        assert L.get_tile()[3] & 16  # replaced by a vertical-stack tile
        with pytest.raises(lbm.LBMError) as ei:
            L.set_tile(1, 1, 4, 0)
        assert ei.value.status == lbm.EINVAL
        with pytest.raises(lbm.LBMError):
            L.set_model(lbm.MODEL_EQUILIBRIUM)
        bad = np.full((12, 16), 0.3)
        bad[3, 4] = 0.0
        with pytest.raises(lbm.LBMError):
            L.set_c2_field(bad)
        L.set_c2_field(None)
        L.set_tile(1, 1, 4, 0)
    with lbm.Lattice(16, 12, 0.7, 0.3, "f32", model=lbm.MODEL_EQUILIBRIUM) as L:
        with pytest.raises(lbm.LBMError):
            L.set_c2_field(np.full((12, 16), 0.3))
