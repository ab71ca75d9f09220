"""Pins of the oracle on nonlinear progressive waves (Sec. 4, Figs. 2-3).

The paper propagated a finite-amplitude sine wave until it steepened towards
a shock (at the distance of Eq. 9) and compared its form with Burgers'
equation. Here the oracle's wave is compared, harmonic by harmonic, with the
exact Cole-Hopf solution of Burgers' equation (tests/burgers.py): the paper's
two waves (c_e = 0.2 and 0.9, nu = 0.01), scaled to lambda = 400 and
u0 = 0.004 so that sigma = k u0 t reaches 1 (the shock) and 1.5 in about
24 000 steps. The bar, 5e-3 u0 for the first three harmonics, covers the
lattice's sound dispersion at these wavelengths (phase-speed errors of
2e-4 ... 2e-3 for harmonics 1-3 at c_e = 0.2, from the linear theory).
"""
import numpy as np
import pytest

import burgers
import oracle
from paper_0707_2437_amd import workloads


@pytest.mark.parametrize("c2", [0.04, 0.81])
def test_harmonics_follow_burgers(c2):
    lam, ny, u0, tau = 400, 3, 0.004, 0.53
    k, nu = 2 * np.pi / lam, (2 * tau - 1) / 6
    o = oracle.Oracle(lam, ny, tau, c2).init(*workloads.simple_wave_fields(lam, ny, c2, u0))
    ts = burgers.shock_time(u0, k)
    for sigma in (1.0, 1.5):
        t = int(round(sigma * ts))
        o.step(t - o.time)
        ux = o.moments()[1]
        got = np.abs(np.fft.rfft(ux[0]) * (2.0 / lam))[1:4]
        want = burgers.harmonics(u0, k, nu, t, 3)
        assert np.max(np.abs(got - want)) < 5e-3 * u0, (sigma, got / u0, want / u0)
        # harmonics grow: the second is a third of the fundamental by sigma = 1
        assert got[1] > 0.3 * got[0]
        # the wave stays one-dimensional
        assert np.max(np.abs(ux - ux[0:1])) == 0.0


def test_burgers_reference_limits():
    """The Cole-Hopf helper against independent closed forms: a short time
    after the start, u0 sin(kx) (to O(t)); the linear limit (small u0),
    u0 exp(-nu k^2 t) sin(kx); and the inviscid limit before the shock,
    Fubini's series b_n = 2 u0 J_n(n sigma) / (n sigma), sigma = k u0 t."""
    from scipy.special import jv

    k = 2 * np.pi / 400
    x = np.arange(0.0, 400.0, 7.0)
    u = burgers.velocity(0.004, k, 0.01, 1.0, x)
    assert np.max(np.abs(u - 0.004 * np.sin(k * x))) < 0.004 * 2 * k * 0.004 * 1.0 + 1e-9
    b = burgers.harmonics(1e-9, k, 0.01, 5000.0, 3)
    assert abs(b[0] / (1e-9 * np.exp(-k * k * 0.01 * 5000)) - 1) < 1e-6 and b[1] < 1e-6 * b[0]
    u0, nu, sigma = 0.004, 2e-4, 0.6
    t = sigma / (k * u0)
    got = burgers.harmonics(u0, k, nu, t, 5) / u0
    n = np.arange(1, 6)
    fubini = 2 * jv(n, n * sigma) / (n * sigma) * np.exp(-(n * k) ** 2 * nu * t)
    assert np.max(np.abs(got - fubini)) < 2e-3, (got, fubini)
