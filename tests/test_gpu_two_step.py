"""The two-step form (LBM_TILE_VSTACK | LBM_TILE_TWO_STEP: two steps of Eq. 5
per launch, the first step's results held in LDS) gives the bits of single
steps: every shape, stored type (FP16 storage included) and store flavour, on lattices that span
several tiles with ragged edges and on lattices smaller than one tile (whose
halo rows and columns are periodic images of the lattice itself), for odd
and even step counts (a lone last step takes the single-step kernel). The
oracle check of the single-step path therefore carries over; one case is
also checked against the oracle directly."""
import numpy as np
import pytest

import oracle
from gpu_util import max_rel_err, smooth_random_state

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_0707_2437_amd as lbm  # noqa: E402

VSTACK, TWO_STEP, NT = 16, 32, 2
SHAPES = [(vx, nw, f) for vx in (1, 2) for nw in (12, 16) for f in (VSTACK | TWO_STEP, VSTACK | TWO_STEP | NT)]
ROWS32 = [(1, 32, VSTACK | TWO_STEP), (1, 32, VSTACK | TWO_STEP | NT)]  # two rows per wave; not FP64


def shapes_for(dtype):
    return SHAPES + ([] if dtype == "f64" else ROWS32)


def run(nx, ny, tau, c2, dtype, steps, fields, tile=None, model=None):
    with lbm.Lattice(nx, ny, tau, c2, dtype) as L:
        if model is not None:
            L.set_model(model)
        if tile:
            L.set_tile(*tile)
        L.init(*fields)
        L.step(steps)
        return L.get_f()


@pytest.mark.parametrize("dtype", ["f64", "f32", "f32s", "f16s"])
@pytest.mark.parametrize("nx,ny", [(3, 3), (5, 4), (7, 3), (65, 3), (130, 77), (300, 41), (257, 129)])
def test_two_step_bitwise_equals_single_steps(dtype, nx, ny):
    fields = smooth_random_state(nx, ny, seed=nx * 31 + ny)
    for steps in (6, 7):
        ref = run(nx, ny, 0.7, 0.45, dtype, steps, fields)
        for vx, nw, f in shapes_for(dtype):
            got = run(nx, ny, 0.7, 0.45, dtype, steps, fields, (vx, nw, 0, f))
            assert np.array_equal(got, ref), (dtype, nx, ny, steps, vx, nw, f)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_two_step_altered_equilibrium_model_bitwise(dtype):
    nx, ny = 200, 90
    fields = smooth_random_state(nx, ny, seed=5)
    ref = run(nx, ny, 0.75, 0.2, dtype, 8, fields, model=lbm.MODEL_EQUILIBRIUM)
    for vx, nw in ((1, 16), (2, 12)):
        got = run(nx, ny, 0.75, 0.2, dtype, 8, fields, (vx, nw, 0, VSTACK | TWO_STEP | NT), model=lbm.MODEL_EQUILIBRIUM)
        assert np.array_equal(got, ref), (dtype, vx, nw)


def test_two_step_parity_with_oracle():
    nx, ny, tau, c2 = 130, 77, 0.8, 0.2
    fields = smooth_random_state(nx, ny, seed=77)
    ref = oracle.Oracle(nx, ny, tau, c2).init(*fields).step(40).get_f()
    for dtype, tol in (("f64", 1e-12), ("f32", 1e-5)):
        got = run(nx, ny, tau, c2, dtype, 40, fields, (2, 16, 0, VSTACK | TWO_STEP | NT))
        assert max_rel_err(got, ref) <= tol, dtype


@pytest.mark.parametrize("dtype", ["f32", "f64", "f16s"])
def test_two_step_full_size_bitwise(dtype):
    """4096 x 4096, the benchmark's lattice: 10 steps (5 two-step launches)
    in the default two-step shapes against 10 single steps."""
    n = 4096
    rng = np.random.default_rng(3)
    rho = 1.0 + 1e-3 * rng.standard_normal((n, n))
    ux = 1e-3 * rng.standard_normal((n, n))
    uy = 1e-3 * rng.standard_normal((n, n))
    single = (4, 8, 0, VSTACK | NT) if dtype == "f16s" else (2, 8, 0, VSTACK | NT)
    ref = run(n, n, 0.6, 0.25, dtype, 10, (rho, ux, uy), single)
    shapes = [(1, 16, VSTACK | TWO_STEP | NT), (2, 16, VSTACK | TWO_STEP | NT)]
    if dtype != "f64":
        shapes.append((1, 32, VSTACK | TWO_STEP))  # two rows per wave (FP16's default)
    for vx, nw, f in shapes:
        got = run(n, n, 0.6, 0.25, dtype, 10, (rho, ux, uy), (vx, nw, 0, f))
        assert np.array_equal(got, ref), (dtype, vx, nw, f)
        del got


def test_two_step_with_inlet_outlet():
    nx, ny = 160, 40
    fields = smooth_random_state(nx, ny, seed=9)
    with lbm.Lattice(nx, ny, 0.7, 0.3, "f32") as L:
        L.set_tile(2, 16, 0, VSTACK | TWO_STEP)
        L.set_x_boundaries(lbm.XBC_INLET_OUTLET, 0.01, 50.0)
        got = L.init(*fields).step(9).get_f()
    with lbm.Lattice(nx, ny, 0.7, 0.3, "f32") as L:
        L.set_x_boundaries(lbm.XBC_INLET_OUTLET, 0.01, 50.0)
        ref = L.init(*fields).step(9).get_f()
    assert np.array_equal(got, ref)



def test_two_step_shape_errors():
    with lbm.Lattice(64, 64, 0.7, 0.3, "f32") as L:
        L.set_tile(1, 32, 0, VSTACK | TWO_STEP)
        for bad in ((4, 16, 0, VSTACK | TWO_STEP), (2, 8, 0, VSTACK | TWO_STEP), (2, 16, 0, TWO_STEP),
                    (2, 16, 0, VSTACK | TWO_STEP | 1), (2, 16, 0, 64 | VSTACK), (2, 32, 0, VSTACK | TWO_STEP)):
            with pytest.raises(lbm.LBMError):
                L.set_tile(*bad)
    with lbm.Lattice(64, 64, 0.7, 0.3, "f64") as L:
        with pytest.raises(lbm.LBMError):
            L.set_tile(1, 32, 0, VSTACK | TWO_STEP)  # 32-row tiles: 4-byte or smaller storage
    with lbm.Lattice(64, 64, 0.7, 0.3, "f16s") as L:  # FP16 storage has the two-step form too
        assert L.get_tile() == (1, 32, 8, VSTACK | TWO_STEP)  # its default
        L.set_tile(2, 16, 0, VSTACK | TWO_STEP)


@pytest.mark.parametrize("dtype", ["f64", "f32", "f32s", "f16s"])
@pytest.mark.parametrize("nx,ny", [(3, 3), (7, 5), (130, 77), (300, 41)])
def test_two_step_c2_field_bitwise(dtype, nx, ny):
    """A c2 field varying in x and y (per-site source coefficients, read once
    per two-step launch for both steps) gives the bits of single steps."""
    fields = smooth_random_state(nx, ny, seed=nx + 7 * ny)
    yy, xx = np.mgrid[0:ny, 0:nx]
    c2 = 0.2 + 0.15 * np.sin(2 * np.pi * xx / nx) * np.cos(2 * np.pi * yy / ny) + 0.001 * xx / nx

    def go(tile):
        with lbm.Lattice(nx, ny, 0.7, 0.3, dtype) as L:
            L.set_c2_field(c2)
            if tile:
                L.set_tile(*tile)
            return L.init(*fields).step(7).get_f()

    ref = go((4, 8, 0, VSTACK | NT) if dtype == "f16s" else (2, 8, 0, VSTACK | NT))
    for vx, nw, f in shapes_for(dtype):
        assert np.array_equal(go((vx, nw, 0, f)), ref), (dtype, nx, ny, vx, nw, f)
    assert np.array_equal(go(None), ref)  # the default shape


def test_march_shape_with_field_takes_the_default():
    with lbm.Lattice(64, 64, 0.7, 0.3, "f32") as L:
        L.set_tile(1, 1, 4, 0)
        L.set_c2_field(np.full((64, 64), 0.3))
        assert L.get_tile()[3] & (VSTACK | TWO_STEP) == VSTACK | TWO_STEP
