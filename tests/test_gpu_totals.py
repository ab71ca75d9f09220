"""Conservation totals of the GPU path: M = sum rho and P = sum rho u (Eq. 3)
of the current state, accumulated in FP64 by the library's fixed-order
reduction, on a state that carries momentum in both directions.

- Against an exact sum of the GPU's own state: the populations the library
  exports (lbm_get_f) summed per component with math.fsum. Only the order of
  the FP64 additions differs, so the totals agree to a few ulps of the sum
  of magnitudes; a swapped or mis-signed component fails by orders of
  magnitude.
- Against the oracle's totals after the same steps: FP64 within 1e-12 of
  the total mass; the FP32 forms within the state difference itself,
  sum over sites of |rho u (GPU) - rho u (oracle)|, computed from the two
  exported states.
"""
import math

import numpy as np
import pytest

import oracle
from gpu_util import smooth_random_state

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_0707_2437_amd as lbm  # noqa: E402

E = np.array([(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)], dtype=np.float64)
NX, NY, TAU, C2, STEPS = 70, 53, 0.7, 0.3, 500


def flowing_state():
    rho, ux, uy = smooth_random_state(NX, NY, seed=11)
    return rho, ux + 0.03, uy - 0.02  # a mean flow: both momentum totals far from zero


def exact_totals(f):
    """(sum rho, sum rho u_x, sum rho u_y) of populations f[9][ny][nx], exactly rounded."""
    return [math.fsum(f.reshape(-1)),
            math.fsum((f * E[:, 0, None, None]).reshape(-1)),
            math.fsum((f * E[:, 1, None, None]).reshape(-1))]


def site_momentum(f):
    return np.tensordot(E[:, 0], f, axes=1), np.tensordot(E[:, 1], f, axes=1)


@pytest.mark.parametrize("dtype", ["f64", "f32", "f32s", "f16s"])
def test_totals_match_exact_sum_and_oracle(dtype):
    rho, ux, uy = flowing_state()
    o = oracle.Oracle(NX, NY, TAU, C2).init(rho, ux, uy)
    with lbm.Lattice(NX, NY, TAU, C2, dtype) as L:
        L.init(rho, ux, uy)
        for steps in (0, STEPS):
            L.step(steps)
            o.step(steps)
            tot = np.asarray(L.totals())
            f = L.get_f()
            ref_f = o.get_f()
            _, _, _, ref_tot = o.moments()
            mass = ref_tot[0]
            assert abs(ref_tot[1]) > 0.01 * mass and abs(ref_tot[2]) > 0.005 * mass  # momentum in both
            # the reduction against an exact sum of the same state
            ex = exact_totals(f)
            scale = float(np.sum(np.abs(f)))
            for k in range(3):
                assert abs(tot[k] - ex[k]) <= 64 * 2.0 ** -52 * scale, (dtype, steps, k, tot[k], ex[k])
            # against the oracle
            if dtype == "f64":
                assert np.all(np.abs(tot - ref_tot) <= 1e-12 * mass), (steps, tot, ref_tot)
            else:
                jx, jy = site_momentum(f)
                rjx, rjy = site_momentum(ref_f)
                bound = [float(np.sum(np.abs(f - ref_f))), float(np.sum(np.abs(jx - rjx))),
                         float(np.sum(np.abs(jy - rjy)))]
                for k in range(3):
                    assert abs(tot[k] - ref_tot[k]) <= bound[k] + 1e-12 * mass, (dtype, steps, k)
    o.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_moment_fields_match_oracle(dtype):
    """rho and u = rho u / rho (Eq. 3) per site, after the same steps."""
    rho, ux, uy = flowing_state()
    o = oracle.Oracle(NX, NY, TAU, C2).init(rho, ux, uy).step(STEPS)
    r_ref, ux_ref, uy_ref, _ = o.moments()
    with lbm.Lattice(NX, NY, TAU, C2, dtype) as L:
        r, vx, vy, _ = L.init(rho, ux, uy).step(STEPS).moments()
    # the bar on f (max relative error tol, all f_i > 0) bounds the moments:
    # |d rho| <= tol rho and |d(rho u)| <= tol rho, so |d u| <= tol (1 + |u|)
    tol = 1e-12 if dtype == "f64" else 1e-5
    assert np.max(np.abs(r - r_ref) / r_ref) <= tol
    umax = max(np.max(np.abs(ux_ref)), np.max(np.abs(uy_ref)))
    assert np.max(np.abs(vx - ux_ref)) <= tol * (1 + umax)
    assert np.max(np.abs(vy - uy_ref)) <= tol * (1 + umax)
