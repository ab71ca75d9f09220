"""Pins of the oracle's Fig. 1 boundaries (an oscillating-density inlet at
x = 0, rho = 1 and u = 0 at the far end; Sec. 4).

The paper measured c_e on this set-up by time of flight and by the ratio of
velocity to density perturbation. The oracle's boundary rule (lbmref.h): the
two boundary columns emit equilibria at rest at rho_in(t) and 1, and the
periodic seam between them is cut. Pinned by:

- the rule itself, population by population, from the weights of Sec. 2
  (at rest feq_i = w_i rho for the forcing model) and the inlet's sine;
- a rest state with a silent inlet stays at rest (to a few ulps: the
  interior relaxes towards its summed density, the boundary emits the
  weights themselves);
- the emitted wave, in its periodic regime, against acoustics: phase speed
  c_e, spatial decay exp(-nu k^2 x / c_e) (temporal decay nu k^2 carried at
  c_e), u / delta rho = c_e / rho0 (a progressive wave, Eq. 8), and the
  time of flight of its front between two probes.
"""
import numpy as np
import pytest

import oracle

W = np.array([4, 1, 1, 1, 1, 0.25, 0.25, 0.25, 0.25]) / 9.0
EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])


def rho_in(t, amp, period):
    return 1.0 + amp * np.sin(2 * np.pi * t / period)


def test_emission_rule_population_by_population():
    """After the step from time t: column 1 holds, in its +x populations, what
    x = 0 emitted (w_i rho_in(t)); column nx - 2 holds in its -x populations
    w_i * 1; across the cut seam column 0 receives w_i rho_in(t) and column
    nx - 1 receives w_i. Several steps, a non-trivial interior."""
    nx, ny, amp, period = 9, 4, 0.05, 7.0
    rng = np.random.default_rng(2)
    o = oracle.Oracle(nx, ny, 0.7, 0.2).set_x_boundaries(oracle.XBC_INLET_OUTLET, amp, period)
    o.init(1 + 0.01 * rng.standard_normal((ny, nx)), 0.01 * rng.standard_normal((ny, nx)), None)
    plus, minus = EX > 0, EX < 0
    for t in range(6):
        o.step(1)
        f = o.get_f()  # f_i(x, t + 1)
        r = rho_in(t, amp, period)
        for y in range(ny):
            assert np.allclose(f[plus, y, 1], W[plus] * r, rtol=0, atol=1e-16)
            assert np.allclose(f[plus, y, 0], W[plus] * r, rtol=0, atol=1e-16)
            assert np.allclose(f[minus, y, nx - 2], W[minus], rtol=0, atol=1e-16)
            assert np.allclose(f[minus, y, nx - 1], W[minus], rtol=0, atol=1e-16)
            # rest populations: what the column emitted to itself
            assert abs(f[0, y, 0] - W[0] * r) <= 1e-16 and abs(f[0, y, nx - 1] - W[0]) <= 1e-16


def test_silent_inlet_keeps_rest_state():
    o = oracle.Oracle(12, 5, 0.8, 0.3).set_x_boundaries(oracle.XBC_INLET_OUTLET, 0.0, 100.0).init()
    f0 = o.get_f()
    o.step(30)
    assert np.max(np.abs(o.get_f() - f0)) <= 4e-16
    assert np.max(np.abs(o.moments()[1])) <= 1e-15


@pytest.mark.parametrize("c2", [0.09, 0.25, 0.64])
def test_emitted_wave_is_a_sound_wave_at_c(c2):
    """Inlet period 250, probes at x = 200 and 400 on a 1200 x 3 lattice,
    tau = 0.6; the window (4 periods after the front has passed both
    probes by 3 periods) ends before the outlet's echo reaches them."""
    nx, ny, tau, T, amp, x1, x2 = 1200, 3, 0.6, 250, 1e-3, 200, 400
    c, w = np.sqrt(c2), 2 * np.pi / T
    k, nu = w / c, (2 * tau - 1) / 6
    t0 = int(x2 / c + 3 * T)
    t1 = t0 + 4 * T
    assert (2 * nx - x2) / c > t1
    o = oracle.Oracle(nx, ny, tau, c2).set_x_boundaries(oracle.XBC_INLET_OUTLET, amp, T).init()
    R, U = np.empty((t1, 2)), np.empty((t1, 2))
    for t in range(t1):
        rho, ux, _, _ = o.moments()
        R[t], U[t] = rho[0, [x1, x2]] - 1, ux[0, [x1, x2]]
        o.step(1)
    ph = np.exp(-1j * w * np.arange(t0, t1))[:, None]
    a, b = (R[t0:] * ph).mean(0), (U[t0:] * ph).mean(0)
    # phase speed (the phase advance between the probes, unwrapped near k dx)
    dphi = np.angle(a[0] / a[1])
    dphi += 2 * np.pi * np.round((k * (x2 - x1) - dphi) / (2 * np.pi))
    assert abs(w * (x2 - x1) / dphi / c - 1) < 5e-3
    # spatial decay of a wave damped at nu k^2 in time and carried at c
    assert abs(-np.log(abs(a[1] / a[0])) / (x2 - x1) / (nu * k * k / c) - 1) < 3e-2
    # a progressive wave: u = c delta rho / rho0, in phase
    for j in range(2):
        assert abs(abs(b[j] / a[j]) / c - 1) < 1e-2
        assert abs(np.angle(b[j] / a[j])) < 6e-2
    # time of flight of the front: first time |delta rho| reaches its
    # periodic-regime amplitude, at each probe
    th = [np.argmax(np.abs(R[:, j]) >= abs(2 * a[j])) for j in range(2)]
    assert abs((x2 - x1) / (th[1] - th[0]) / c - 1) < 3e-2


def test_rejections():
    o = oracle.Oracle(5, 3, 0.7, 0.3)
    for args in [(1, 1.0, 10.0), (1, -1.5, 10.0), (1, 0.1, 0.0), (1, 0.1, np.nan), (2, 0.1, 10.0)]:
        with pytest.raises(oracle.lbmref.OracleError):
            o.set_x_boundaries(*args)
    with pytest.raises(oracle.lbmref.OracleError):
        oracle.Oracle(4, 3, 0.7, 0.3).set_x_boundaries(oracle.XBC_INLET_OUTLET, 0.1, 10.0)
    o.set_x_boundaries(oracle.XBC_INLET_OUTLET, 0.1, 10.0).set_x_boundaries(oracle.XBC_PERIODIC)
