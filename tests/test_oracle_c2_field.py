"""Pins of the oracle's c2 field: a speed of sound that varies in space.

The paper keeps alpha constant but notes (Sec. 5) that nothing requires it:
alpha may vary within a simulation, e.g. for an acoustic lens or a
temperature gradient. The oracle takes a per-site c_e^2 and uses
alpha(x) = 1/3 - c2(x) in the source term of Eq. 5 at that site. Pinned by:

- one step equal to an exact-rational brute force with per-site alpha;
- a uniform field equal to the scalar lattice, bitwise;
- the momentum balance: total momentum now changes by sum_x alpha(x) G(x)
  per step (the force no longer telescopes), total mass is conserved;
- acoustics of an interface between two sound speeds (the linearised
  equations give d_tt rho = d_x (c^2(x) d_x rho): rho and the mass flux are
  continuous): a pulse meeting it is reflected with amplitude
  (c_A - c_B)/(c_A + c_B) and its transmitted part carries 2 c_B/(c_A + c_B)
  of the mass and moves at c_B;
- rejection of non-positive entries and of the equilibrium model.
"""
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle
from test_oracle_pins import brute_step


@pytest.mark.parametrize("nx,ny", [(3, 3), (4, 5), (5, 3)])
def test_one_step_per_site_alpha_matches_exact_brute_force(nx, ny):
    rng = np.random.default_rng(77 * nx + ny)
    f = [[[Fr(int(rng.integers(200, 900)), 4096) for _ in range(nx)] for _ in range(ny)] for _ in range(9)]
    # dyadic c2 in (0, 1): exact in FP64, and 1/3 - c2 is then held to FP64 rounding
    c2 = [[Fr(int(rng.integers(8, 120)), 128) for _ in range(nx)] for _ in range(ny)]
    o = oracle.Oracle(nx, ny, 0.8, 0.25)
    o.set_c2_field(np.array([[float(v) for v in row] for row in c2]))
    o.set_f(np.array([[[float(v) for v in row] for row in plane] for plane in f]))
    o.step(1)
    got = o.get_f()
    want = brute_step(f, nx, ny, Fr(0.8), c2)
    for i in range(9):
        for y in range(ny):
            for x in range(nx):
                assert abs(Fr(got[i, y, x]) - want[i][y][x]) <= Fr(2, 10**15), (i, y, x)


def _state(nx, ny, seed):
    rng = np.random.default_rng(seed)
    y, x = np.mgrid[0:ny, 0:nx]
    rho = 1 + 0.01 * np.sin(2 * np.pi * x / nx) * np.cos(2 * np.pi * y / ny) + 1e-3 * rng.standard_normal((ny, nx))
    return rho, 0.02 * rng.standard_normal((ny, nx)), 0.02 * rng.standard_normal((ny, nx))


def test_uniform_field_is_the_scalar_lattice_bitwise():
    nx, ny = 21, 13
    fields = _state(nx, ny, 3)
    a = oracle.Oracle(nx, ny, 0.7, 0.2).init(*fields).step(40)
    b = oracle.Oracle(nx, ny, 0.7, 0.2).set_c2_field(np.full((ny, nx), 0.2)).init(*fields).step(40)
    assert np.array_equal(a.get_f(), b.get_f())
    # removing the field restores the lattice's own c2
    c = oracle.Oracle(nx, ny, 0.7, 0.2).set_c2_field(np.full((ny, nx), 0.5)).set_c2_field(None)
    assert np.array_equal(c.init(*fields).step(40).get_f(), a.get_f())


def test_momentum_balance_and_mass():
    """Streaming and BGK conserve mass and momentum, the source has no mass and
    its momentum is alpha(x) G(x) at each site: sum_x of it is the change of
    the total momentum over one step (computed here from the moments alone)."""
    nx, ny = 24, 17
    y, x = np.mgrid[0:ny, 0:nx]
    c2 = 0.2 + 0.15 * np.sin(2 * np.pi * x / nx) + 0.05 * np.cos(2 * np.pi * y / ny)
    o = oracle.Oracle(nx, ny, 0.7, 0.3).set_c2_field(c2).init(*_state(nx, ny, 9))
    alpha = 1.0 / 3.0 - c2
    for _ in range(5):
        rho, _, _, t0 = o.moments()
        gx = (np.roll(rho, -1, axis=1) - np.roll(rho, 1, axis=1)) / 2
        gy = (np.roll(rho, -1, axis=0) - np.roll(rho, 1, axis=0)) / 2
        o.step(1)
        t1 = o.moments()[3]
        assert abs(t1[0] - t0[0]) < 1e-12 * t0[0]
        assert abs((t1[1] - t0[1]) - (alpha * gx).sum()) < 1e-13
        assert abs((t1[2] - t0[2]) - (alpha * gy).sum()) < 1e-13
        # the balance is not trivially zero here
        assert abs((alpha * gx).sum()) > 1e-6


@pytest.mark.parametrize("cB2", [0.09, 0.64])
def test_interface_reflection_and_transmission(cB2):
    """A right-going Gaussian pulse (delta rho = u / c_A) in a region of sound
    speed c_A meets a sharp interface to c_B. After it has split: the
    reflected pulse carries (c_A - c_B)/(c_A + c_B) of the incident mass, the
    transmitted one 2 c_B/(c_A + c_B), and the transmitted one moves at c_B."""
    cA2, nx, ny, x0, xi, sigma, tau, eps = 0.25, 1400, 3, 500, 800, 12.0, 0.55, 1e-4
    cA, cB = np.sqrt(cA2), np.sqrt(cB2)
    x = np.arange(nx)[None, :] * np.ones((ny, 1))
    g = np.exp(-0.5 * ((x - x0) / sigma) ** 2)
    o = oracle.Oracle(nx, ny, tau, cA2).set_c2_field(np.where(x < xi, cA2, cB2))
    o.init(rho=1 + eps * g, ux=cA * eps * g)
    T = int(round(450 / cA))
    o.step(T)
    r = o.moments()[0][0] - 1
    assert np.allclose(o.moments()[0], o.moments()[0][0:1, :], rtol=0, atol=1e-15)  # stays 1-D
    a_inc = eps * g[0].sum()
    t_split = T - (xi - x0) / cA
    xr, xt = xi - cA * t_split, xi + cB * t_split
    wr = slice(int(xr - 8 * sigma), int(xr + 8 * sigma))
    wt = slice(int(xt - 8 * sigma * cB / cA), int(xt + 8 * sigma * cB / cA))
    R, Tm = r[wr].sum() / a_inc, r[wt].sum() / a_inc
    assert abs(R - (cA - cB) / (cA + cB)) < 1e-3
    assert abs(Tm - 2 * cB / (cA + cB)) < 1e-3
    xs = np.arange(nx)
    centre = (xs[wt] * r[wt]).sum() / r[wt].sum()
    assert abs((centre - xi) / t_split / cB - 1) < 3e-3


def test_rejections():
    o = oracle.Oracle(6, 5, 0.7, 0.3)
    for bad in (0.0, -0.1, np.nan, np.inf):
        c2 = np.full((5, 6), 0.3)
        c2[2, 3] = bad
        with pytest.raises(oracle.lbmref.OracleError):
            o.set_c2_field(c2)
    e = oracle.Oracle(6, 5, 0.7, 0.3, model=oracle.MODEL_EQUILIBRIUM)
    with pytest.raises(oracle.lbmref.OracleError):
        e.set_c2_field(np.full((5, 6), 0.3))
    o.set_c2_field(np.full((5, 6), 0.3))
    with pytest.raises(oracle.lbmref.OracleError):
        o._check(o.lib.lbmref_set_model(o._h, oracle.MODEL_EQUILIBRIUM), "set_model")
