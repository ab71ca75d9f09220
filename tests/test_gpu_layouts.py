"""The two storage layouts and the largest lattices, on the GPU through the C
ABI. A lattice is stored row-interleaved when its whole buffer fits the
kernels' 32-bit byte offsets (about 119 M sites in FP32, 60 M in FP64), and
plane-major beyond that (each plane must fit). LBM_LAYOUT=soa forces the
plane-major layout at lbm_create, so that small lattices can test it. The
largest lattices take the default shape: two steps per launch (and a lone
last step) for FP32 and FP64."""
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
TILES = [(2, 8, 0, 18), (1, 8, 0, 18), (4, 8, 0, 16), (2, 16, 0, 18), (1, 1, 1, 0), (2, 4, 8, 15),
         (2, 16, 0, 50), (1, 12, 0, 48)]  # the last two: two steps per launch


def run(nx, ny, dtype, fields, tile, steps=30):
    with lbm.Lattice(nx, ny, 0.7, 0.3, dtype) as L:
        L.set_tile(*tile)
        return L.init(*fields).step(steps).get_f()


@pytest.mark.parametrize("dtype", ["f64", "f32", "f32s", "f16s"])
def test_plane_major_layout_bitwise_equal(dtype, monkeypatch):
    for nx, ny in [(397, 131), (130, 9), (5, 7)]:
        fields = smooth_random_state(nx, ny, seed=nx + ny)
        ref = [run(nx, ny, dtype, fields, t) for t in TILES[:2]]
        monkeypatch.setenv("LBM_LAYOUT", "soa")
        outs = [run(nx, ny, dtype, fields, t) for t in TILES]
        monkeypatch.delenv("LBM_LAYOUT")
        for t, o in zip(TILES, outs):
            assert np.array_equal(o, ref[0]), (nx, ny, t)
        fr = oracle.Oracle(nx, ny, 0.7, 0.3).init(*fields).step(30).get_f()
        assert max_rel_err(ref[0], fr) <= TOL[dtype]


def _fields(nx, ny, x, y, m=np):
    """A plane wave in x plus a weaker one in y (both periodic), at rest in y;
    m is the array module (numpy on the host, torch on the device)."""
    rho = 1.0 + 1e-3 * m.sin(2 * np.pi * x / nx) + 5e-4 * m.cos(2 * np.pi * y / ny)
    ux = 0.5e-3 * m.sin(2 * np.pi * x / nx) + 0 * y
    return rho, ux


@pytest.mark.parametrize("dtype,nx,ny", [("f32", 32768, 32703), ("f64", 32768, 16367)])
def test_largest_lattice(dtype, nx, ny):
    """The largest lattice the library accepts (plane-major, 77 GB of HBM):
    sampled sites, edges included, against the oracle on a periodic window
    of half-width 2 n + 2 (exact after n steps), and conservation."""
    steps = 3
    dev = torch.device("cuda")
    y = torch.arange(ny, dtype=torch.float64, device=dev)[:, None]
    x = torch.arange(nx, dtype=torch.float64, device=dev)[None, :]
    rho, ux = _fields(nx, ny, x, y, torch)
    rho, ux = rho.contiguous().view(-1), ux.expand(ny, nx).contiguous().view(-1)
    xs = np.array([0, nx - 1, 0, nx - 1, 1, nx // 2, 12345, 32767])
    ys = np.array([0, ny - 1, ny - 1, 0, 1, ny // 2, 23456 % ny, 7])
    torch.cuda.synchronize()  # the fields are written on torch's stream, read on the lattice's
    with lbm.Lattice(nx, ny, 0.8, 0.25, dtype) as L:
        L.init_device(rho, ux, None)
        t0 = L.totals()  # synchronises the lattice's stream: the fields are read
        del rho, ux
        got = L.step(steps).sample_f(xs, ys)
        t1 = L.totals()
    torch.cuda.empty_cache()
    R = 2 * steps + 2
    want = []
    for xc, yc in zip(xs, ys):
        wy = (yc + np.arange(-R, R + 1)) % ny
        wx = (xc + np.arange(-R, R + 1)) % nx
        r, u = _fields(nx, ny, wx[None, :].astype(float), wy[:, None].astype(float))
        o = oracle.Oracle(2 * R + 1, 2 * R + 1, 0.8, 0.25).init(r, np.broadcast_to(u, r.shape), None)
        want.append(o.step(steps).get_f()[:, R, R])
    err = max_rel_err(got, np.array(want))
    print(f"largest {dtype} lattice {nx} x {ny}: max rel err over {len(xs)} sites = {err:.3e}")
    assert err <= TOL[dtype]
    assert abs(t1[0] - t0[0]) <= 1e-9 * t0[0]
