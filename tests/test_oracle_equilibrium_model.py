"""Pins of the oracle's altered-equilibrium model.

The paper (Sec. 3, opening) names the other route to a variable speed of
sound: change the equilibrium, i.e. the share of rest and moving particles,
instead of adding a force. On D2Q9 the oracle's form of it
(lbmref_equilibrium_c2) is pinned here by what fixes it independently of its
code:

- its moments are exactly rho, rho u and c^2 rho I + rho u u, and c^2 = 1/3
  gives Eq. 2;
- small-amplitude evolution equals the linear theory of the scheme
  (tests/linear_theory.py, model=1), which has sound speed c;
- a progressive wave moves at c;
- shear waves decay with nu = (2 tau - 1)/6 (the change touches only the
  isotropic part of the momentum flux);
- sound decays at 1.5 (1 - c^2) nu k^2: the first-order stress keeps the
  c-independent third moment of Eq. 2, so its trace part no longer cancels
  and the effective longitudinal viscosity is 3 (1 - c^2) nu (nu k^2 at
  c^2 = 1/3, as for the paper's model at every c);
- mass and momentum are conserved and the rest state stays at rest;
- c^2 >= 3/5 is rejected (the rest population would not be positive).
"""
from fractions import Fraction

import numpy as np
import pytest

import linear_theory as lt
import oracle

E = [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)]


def fourier(field, k, axis):
    n = field.shape[axis]
    ph = np.exp(-1j * k * np.arange(n))
    if axis == 1:
        return 2.0 * (field * ph[None, :]).mean()
    return 2.0 * (field * ph[:, None]).mean()


@pytest.mark.parametrize("rho,ux,uy,c2", [(1.25, 0.0625, -0.03125, 0.25), (0.75, -0.125, 0.1875, 0.0625),
                                          (1.0, 0.0, 0.0, 0.5), (1.5, 0.25, 0.125, 0.125)])
def test_moments_are_exact(rho, ux, uy, c2):
    """Sum feq = rho, sum feq e = rho u, sum feq e e = c^2 rho I + rho u u
    (exact rational identities; the inputs are dyadic)."""
    feq = oracle.equilibrium_c2(c2, rho, ux, uy)
    f = [Fraction(v) for v in feq]
    R, U, V, C = Fraction(rho), Fraction(ux), Fraction(uy), Fraction(c2)
    m0 = sum(f)
    mx = sum(fi * e[0] for fi, e in zip(f, E))
    my = sum(fi * e[1] for fi, e in zip(f, E))
    pxx = sum(fi * e[0] * e[0] for fi, e in zip(f, E))
    pxy = sum(fi * e[0] * e[1] for fi, e in zip(f, E))
    pyy = sum(fi * e[1] * e[1] for fi, e in zip(f, E))
    tol = Fraction(1, 10 ** 15)
    assert abs(m0 - R) <= tol
    assert abs(mx - R * U) <= tol and abs(my - R * V) <= tol
    assert abs(pxx - (C * R + R * U * U)) <= tol
    assert abs(pyy - (C * R + R * V * V)) <= tol
    assert abs(pxy - R * U * V) <= tol


def test_one_third_gives_eq2():
    for rho, ux, uy in [(1.0, 0.0, 0.0), (1.1, 0.05, -0.02), (0.9, -0.1, 0.07)]:
        assert np.allclose(oracle.equilibrium_c2(1.0 / 3.0, rho, ux, uy), oracle.equilibrium(rho, ux, uy),
                           rtol=0, atol=1e-15)  # feq_0 = rho - sum of eight terms: a few ulps


@pytest.mark.parametrize("c2", [0.2, 0.45])
def test_follows_linear_theory(c2):
    """64 x 64, tau = 0.8, rho = 1 + 1e-3 sin(2 pi x / 64): equal to the
    linear prediction of the model to O(eps^2)."""
    nx = ny = 64
    eps, tau = 1e-3, 0.8
    x = np.arange(nx)[None, :] * np.ones((ny, 1))
    o = oracle.Oracle(nx, ny, tau, c2, model=oracle.MODEL_EQUILIBRIUM).init(rho=1 + eps * np.sin(2 * np.pi * x / nx))
    for t in (100, 500):
        o.step(t - o.time)
        rho, ux, uy, _ = o.moments()
        r_lin, jx_lin, _ = lt.evolve_fields(eps, 2 * np.pi / nx, 0.0, nx, ny, tau, c2, t, model=1)
        assert np.max(np.abs((rho - 1) - r_lin)) < 3e-6, t
        assert np.max(np.abs(ux - jx_lin)) < 3e-6, t
        assert np.max(np.abs(uy)) < 1e-15


@pytest.mark.parametrize("c2", [0.1, 0.25, 0.45])
def test_sound_speed_is_c(c2):
    """A right-going wave (delta rho / rho0 = u / c) moves at c: from the
    phase of its Fourier component, and from the linear theory's eigenvalue."""
    L, ny, eps, tau, T = 256, 3, 1e-5, 0.55, 100  # k c T < pi: no phase wrap
    k = 2 * np.pi / L
    c = np.sqrt(c2)
    x = np.arange(L)[None, :] * np.ones((ny, 1))
    s = np.sin(k * x)
    o = oracle.Oracle(L, ny, tau, c2, model=oracle.MODEL_EQUILIBRIUM).init(rho=1 + eps * s, ux=c * eps * s)
    a0 = fourier(o.moments()[0] - 1, k, 1)
    o.step(T)
    a1 = fourier(o.moments()[0] - 1, k, 1)
    speed = -np.angle(a1 / a0) / (k * T)
    assert abs(speed / c - 1) < 2e-3
    lam = lt.acoustic_eigs(k, 0.0, tau, c2, model=1)
    assert abs(np.max(np.abs(np.angle(lam))) / (k * c) - 1) < 2e-3


@pytest.mark.parametrize("c2", [0.1, 0.5])
def test_shear_viscosity_unchanged(c2):
    tau, L, nx, U, t = 0.8, 128, 3, 1e-6, 2000
    k = 2 * np.pi / L
    y = np.arange(L)[:, None] * np.ones((1, nx))
    o = oracle.Oracle(nx, L, tau, c2, model=oracle.MODEL_EQUILIBRIUM).init(ux=U * np.sin(k * y))
    a0 = abs(fourier(o.moments()[1], k, 0))
    o.step(t)
    nu_meas = -np.log(abs(fourier(o.moments()[1], k, 0)) / a0) / (k * k * t)
    assert abs(nu_meas / ((2 * tau - 1) / 6) - 1) < 1e-3


@pytest.mark.parametrize("c2", [0.1, 0.25, 0.5])
def test_sound_decay_closed_form(c2):
    """Acoustic energy c^2 |rho_k|^2 + |u_k|^2 of a progressive wave decays as
    exp(-2 Gamma T), Gamma = 1.5 (1 - c^2) nu k^2 (Chapman-Enskog closed
    form; the energy is insensitive to the weak counter-running wave the
    equilibrium start excites). Also checked against the linear theory."""
    L, ny, eps, tau, T = 128, 3, 1e-6, 0.8, 2000
    nu = (2 * tau - 1) / 6
    k = 2 * np.pi / L
    c = np.sqrt(c2)
    x = np.arange(L)[None, :] * np.ones((ny, 1))
    s = np.sin(k * x)
    o = oracle.Oracle(L, ny, tau, c2, model=oracle.MODEL_EQUILIBRIUM).init(rho=1 + eps * s, ux=c * eps * s)

    def energy():
        rho, ux, _, _ = o.moments()
        return c2 * abs(fourier(rho - 1, k, 1)) ** 2 + abs(fourier(ux, k, 1)) ** 2

    e0 = energy()
    o.step(T)
    gamma = -np.log(energy() / e0) / (2 * k * k * T)
    assert abs(gamma / (1.5 * (1 - c2) * nu) - 1) < 2e-3
    kl = 2 * np.pi / 512
    lam = lt.acoustic_eigs(kl, 0.0, tau, c2, model=1)
    lam = lam[np.abs(np.angle(lam)) > 0.5 * c * kl]  # the sound pair
    assert len(lam) == 2
    assert np.allclose(-np.log(np.abs(lam)) / (kl * kl), 1.5 * (1 - c2) * nu, rtol=1e-3)


def test_conservation_and_rest_state():
    nx, ny = 24, 17
    rng = np.random.default_rng(5)
    y, x = np.mgrid[0:ny, 0:nx]
    rho = 1 + 0.01 * np.sin(2 * np.pi * x / nx) * np.cos(2 * np.pi * y / ny) + 1e-3 * rng.standard_normal((ny, nx))
    ux = 0.02 * rng.standard_normal((ny, nx))
    uy = 0.02 * rng.standard_normal((ny, nx))
    o = oracle.Oracle(nx, ny, 0.7, 0.3, model=oracle.MODEL_EQUILIBRIUM).init(rho, ux, uy)
    t0 = o.moments()[3]
    o.step(50)
    t1 = o.moments()[3]
    assert abs(t1[0] - t0[0]) < 1e-12 * t0[0]
    assert abs(t1[1] - t0[1]) < 1e-12 * t0[0] and abs(t1[2] - t0[2]) < 1e-12 * t0[0]
    r = oracle.Oracle(9, 7, 0.6, 0.2, model=oracle.MODEL_EQUILIBRIUM).init()
    f0 = r.get_f()
    r.step(20)
    assert np.array_equal(r.get_f(), f0)
    assert f0[0, 0, 0] == pytest.approx(1 - 5 * 0.2 / 3, abs=1e-15)


def test_rejects_c2_from_three_fifths():
    with pytest.raises(oracle.lbmref.OracleError):
        oracle.Oracle(8, 8, 0.7, 0.6, model=oracle.MODEL_EQUILIBRIUM)
    oracle.Oracle(8, 8, 0.7, 0.59, model=oracle.MODEL_EQUILIBRIUM)
