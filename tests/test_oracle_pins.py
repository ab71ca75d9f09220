"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Exact-arithmetic checks (Python fractions) of the lattice constants (Sec. 2),
the equilibrium moments (Eq. 2, 3), the source moments (Eq. 5) and the
c_e^2 <-> alpha map (Eq. 8); one step on tiny grids against an exact
brute force; conservation, the rest state, and the paper's printed numbers.
"""
from fractions import Fraction as Fr
import itertools
import json
import math
import os

import numpy as np
import pytest

import oracle

# Link vectors evaluated by hand from the formulas of Sec. 2:
# e_i = (cos, sin)[pi(i-1)/2] for i = 1..4; sqrt(2)(cos, sin)[pi(i-9/2)/2] for 5..8.
E_PAPER = [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)]
W_PAPER = [Fr(4, 9)] + [Fr(1, 9)] * 4 + [Fr(1, 36)] * 4


# ---------------------------------------------------------------- P1 ----
def test_lattice_constants_match_paper_formulas():
    e, w = oracle.lattice()
    assert [tuple(v) for v in e.tolist()] == E_PAPER
    for wi, wp in zip(w, W_PAPER):
        assert wi == float(wp)  # the double nearest the paper's rational weight


def test_lattice_moment_identities_exact():
    e, w = E_PAPER, W_PAPER
    assert sum(w) == 1
    for a in range(2):
        assert sum(wi * ei[a] for wi, ei in zip(w, e)) == 0
    for a, b in itertools.product(range(2), repeat=2):
        assert sum(wi * ei[a] * ei[b] for wi, ei in zip(w, e)) == (Fr(1, 3) if a == b else 0)
    # fourth-order isotropy: sum w e_a e_b e_c e_d = (d_ab d_cd + d_ac d_bd + d_ad d_bc)/9
    d = lambda i, j: 1 if i == j else 0
    for a, b, c, dd in itertools.product(range(2), repeat=4):
        lhs = sum(wi * ei[a] * ei[b] * ei[c] * ei[dd] for wi, ei in zip(w, e))
        assert lhs == Fr(d(a, b) * d(c, dd) + d(a, c) * d(b, dd) + d(a, dd) * d(b, c), 9)


# ---------------------------------------------------------------- P2 ----
DYADIC_STATES = [(Fr(r, 8), Fr(ux, 64), Fr(uy, 64))
                 for r in (6, 8, 9, 13) for ux in (-5, 0, 3) for uy in (-2, 0, 7)]


@pytest.mark.parametrize("rho,ux,uy", DYADIC_STATES)
def test_equilibrium_moments(rho, ux, uy):
    """sum feq = rho, sum feq e = rho u, sum feq e e = rho/3 I + rho u u (Eq. 2, 3)."""
    feq = [Fr(v) for v in oracle.equilibrium(float(rho), float(ux), float(uy))]
    u = (ux, uy)
    tol = Fr(1, 10**15)
    assert abs(sum(feq) - rho) <= tol * rho
    for a in range(2):
        assert abs(sum(fi * ei[a] for fi, ei in zip(feq, E_PAPER)) - rho * u[a]) <= tol * rho
    for a, b in itertools.product(range(2), repeat=2):
        m2 = sum(fi * ei[a] * ei[b] for fi, ei in zip(feq, E_PAPER))
        want = rho * u[a] * u[b] + (rho / 3 if a == b else 0)
        assert abs(m2 - want) <= tol * rho


# ---------------------------------------------------------------- P3 ----
@pytest.mark.parametrize("c2", [0.04, 0.2, 1.0 / 3.0, 0.81, 1.1])
@pytest.mark.parametrize("gx,gy", [(1e-3, 0.0), (0.0, -2.5e-4), (3e-4, 7e-5)])
def test_source_moments(c2, gx, gy):
    """Source of Eq. 5: zeroth moment 0, first moment alpha grad rho, second 0.

    With Eq. 2's second moment rho/3 I + rho u u, the momentum flux the scheme
    realises is (1/3 - alpha) rho I + rho u u = c2 rho I + rho u u (Eq. 6-8)."""
    al = oracle.alpha(c2)
    s = [Fr(v) for v in oracle.source(al, gx, gy)]
    assert sum(s) == 0
    g = (Fr(gx), Fr(gy))
    for a in range(2):
        m1 = sum(si * ei[a] for si, ei in zip(s, E_PAPER))
        assert abs(m1 - Fr(al) * g[a]) <= Fr(1, 10**15) * abs(Fr(al) * g[a]) + Fr(1, 10**30)
    for a, b in itertools.product(range(2), repeat=2):
        assert sum(si * ei[a] * ei[b] for si, ei in zip(s, E_PAPER)) == 0
    # pressure coefficient of the realised flux is c2
    assert abs((1.0 / 3.0 - al) - c2) <= 4 * np.finfo(float).eps * max(c2, 1.0 / 3.0)


def test_standard_case_has_zero_forcing():
    """c2 = 1/3 is the standard model: alpha == 0 and the source vanishes."""
    assert oracle.alpha(1.0 / 3.0) == 0.0
    assert np.all(oracle.source(oracle.alpha(1.0 / 3.0), 0.3, -0.2) == 0.0)


# ---------------------------------------------------------------- P4 ----
def brute_step(f, nx, ny, tau, c2):
    """One step of Eq. 5 in exact rationals, written in pull form:
    f_i(x, t+1) = f*_i(x - e_i, t), f* = f - (f - feq)/tau + 3 w alpha grad(rho).e.
    c2 is one number, or a per-site grid c2[y][x] (alpha(x) = 1/3 - c2[y][x])."""
    def alpha_at(y, x):
        return Fr(1, 3) - (c2[y][x] if isinstance(c2, list) else c2)
    rho = [[sum(f[i][y][x] for i in range(9)) for x in range(nx)] for y in range(ny)]
    jx = [[sum(f[i][y][x] * E_PAPER[i][0] for i in range(9)) for x in range(nx)] for y in range(ny)]
    jy = [[sum(f[i][y][x] * E_PAPER[i][1] for i in range(9)) for x in range(nx)] for y in range(ny)]
    fstar = [[[None] * nx for _ in range(ny)] for _ in range(9)]
    for y in range(ny):
        for x in range(nx):
            r = rho[y][x]
            ux, uy = jx[y][x] / r, jy[y][x] / r
            gx = (rho[y][(x + 1) % nx] - rho[y][(x - 1) % nx]) / 2
            gy = (rho[(y + 1) % ny][x] - rho[(y - 1) % ny][x]) / 2
            for i, (ex, ey) in enumerate(E_PAPER):
                eu = ex * ux + ey * uy
                feq = W_PAPER[i] * r * (1 + 3 * eu + Fr(9, 2) * eu * eu - Fr(3, 2) * (ux * ux + uy * uy))
                src = 3 * W_PAPER[i] * alpha_at(y, x) * (ex * gx + ey * gy)
                fstar[i][y][x] = f[i][y][x] - (f[i][y][x] - feq) / tau + src
    return [[[fstar[i][(y - E_PAPER[i][1]) % ny][(x - E_PAPER[i][0]) % nx] for x in range(nx)]
             for y in range(ny)] for i in range(9)]


@pytest.mark.parametrize("nx,ny", [(3, 3), (4, 5), (5, 3)])
def test_one_step_matches_exact_brute_force(nx, ny):
    rng = np.random.default_rng(1000 * nx + ny)
    tau_d, c2_d = 0.8, 0.2
    # start from a non-equilibrium state with dyadic entries (exact in FP64)
    f = [[[Fr(int(rng.integers(200, 900)), 4096) for _ in range(nx)] for _ in range(ny)] for _ in range(9)]
    o = oracle.Oracle(nx, ny, tau_d, c2_d)
    o.set_f(np.array([[[float(v) for v in row] for row in plane] for plane in f]))
    o.step(1)
    got = o.get_f()
    want = brute_step(f, nx, ny, Fr(tau_d), Fr(c2_d))
    # The terms of f* are O(0.1 - 1) and may cancel, so the FP64 result is held
    # to a few units in the last place of those terms, not of f* itself.
    for i in range(9):
        for y in range(ny):
            for x in range(nx):
                w = want[i][y][x]
                assert abs(Fr(got[i, y, x]) - w) <= Fr(2, 10**15), (i, y, x)


# ---------------------------------------------------------------- P5 ----
def _c1_rho(nx=64, ny=64):
    x = np.arange(nx)[None, :] * np.ones((ny, 1))
    return 1.0 + 1e-3 * np.sin(2 * np.pi * x / nx)


@pytest.mark.parametrize("c2", [1.0 / 3.0, 0.2])
def test_conservation_c1(c2):
    """Mass and momentum are conserved: BGK conserves them, the source has zero
    mass and its momentum alpha*grad(rho) telescopes to zero on a periodic grid."""
    o = oracle.Oracle(64, 64, 0.8, c2).init(rho=_c1_rho())
    _, _, _, t0 = o.moments()
    o.step(1000)
    _, _, _, t1 = o.moments()
    assert abs(t1[0] - t0[0]) <= 1e-12 * t0[0]
    assert abs(t1[1]) <= 1e-12 * t0[0] and abs(t1[2]) <= 1e-12 * t0[0]


def test_conservation_nonlinear_2d():
    nx, ny = 23, 17
    rng = np.random.default_rng(5)
    y, x = np.mgrid[0:ny, 0:nx]
    rho = 1 + 0.05 * np.exp(-((x - 11) ** 2 + (y - 8) ** 2) / 8.0) + 0.01 * rng.standard_normal((ny, nx))
    ux = 0.03 * rng.standard_normal((ny, nx))
    uy = 0.03 * rng.standard_normal((ny, nx))
    o = oracle.Oracle(nx, ny, 0.7, 0.5).init(rho, ux, uy)
    _, _, _, t0 = o.moments()
    o.step(300)
    _, _, _, t1 = o.moments()
    assert np.all(np.abs(t1 - t0) <= 1e-12 * t0[0])


def _site_values_in(lattice_shape, seq, plane):
    """Populations of a state whose only nonzero population is plane `plane`,
    holding seq[s] at site s in row-major order (the order of the totals)."""
    ny, nx = lattice_shape
    f = np.zeros((9, ny, nx))
    f[plane].reshape(-1)[: len(seq)] = seq
    return f


# Site values whose exact sum is 2 while summing them in order in FP64 gives
# 0: 1 + 2^60 rounds to 2^60 (a small term lost against a larger running
# sum), 2^60 + 1 again, and -2^60 cancels. A compensated sum keeps both lost
# ones; each of its two branches is taken (the running sum smaller, then
# larger, than the term).
CANCELLING = [1.0, 2.0 ** 60, 1.0, -(2.0 ** 60)]


@pytest.mark.parametrize("plane, component", [(0, (0,)), (1, (0, 1)), (2, (0, 2)), (3, (0, 1))])
def test_totals_are_the_exact_sum_of_site_values(plane, component):
    """The totals M = sum rho, P = sum rho u (Eq. 3) are compensated sums in
    row-major site order: on site values where a plain FP64 sum loses every
    small term, they equal the exactly rounded sum (math.fsum). A state with
    one nonzero plane i gives rho = f_i and rho u = f_i e_i at every site."""
    shape = (3, 4)
    exact = math.fsum(CANCELLING)
    assert exact == 2.0 and sum(CANCELLING) == 0.0  # the case is sensitive
    e = E_PAPER[plane]
    expect = [exact, exact * e[0], exact * e[1]]
    for order in (CANCELLING, CANCELLING[::-1], [2.0 ** 60, 1.0, 1.0, -(2.0 ** 60)]):
        o = oracle.Oracle(shape[1], shape[0], 0.8, 0.2).set_f(_site_values_in(shape, order, plane))
        _, _, _, tot = o.moments(check=False)
        assert list(tot) == expect, (plane, order, tot)


# ---------------------------------------------------------------- P6 ----
@pytest.mark.parametrize("rho0", [1.0, 1.3])
def test_rest_state_stays_at_rest_bitwise(rho0):
    """A uniform state at rest stays uniform and at rest: u == 0 and every site
    equal, bitwise. f itself may move by an ulp once, because the FP64 weights
    sum to 1 + 2^-52, not to 1."""
    o = oracle.Oracle(7, 5, 0.6, 0.81).init(rho=np.full((5, 7), rho0))
    f0 = o.get_f()
    o.step(50)
    f1 = o.get_f()
    assert np.all(f1 == f1[:, :1, :1])
    assert np.all(np.abs(f1 - f0) <= 2 * np.spacing(f0))
    rho, ux, uy, _ = o.moments()
    assert np.all(ux == 0.0) and np.all(uy == 0.0)
    assert np.all(rho == rho[0, 0])


# ---------------------------------------------------------------- P11 ---
GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.json")))


def test_paper_printed_numbers():
    """The paper's printed alpha <-> c_e pairs (Eq. 8), the shock distances of
    Eq. 9 and the nu <-> tau pairs of Eq. 4, against the oracle's alpha(c2)."""
    ce = lambda a: math.sqrt(1.0 / 3.0 - a)
    g = GOLDEN["sound_speed_vs_alpha"]
    (a1, c1), (a2, c2) = g["pairs"]
    assert abs(ce(a1) - c1) < 5e-4 and abs(ce(a2) - c2) < 5e-5
    assert abs(ce(a2) / ce(a1) - g["printed_ratio"]) < 1e-2
    for a, c in GOLDEN["sound_speed_limits"]["pairs"]:
        assert abs(ce(a) - c) < 1e-15
    # the oracle's alpha(c2) is the inverse of Eq. 8
    for a in (a1, a2, -0.6, -0.65, 0.0):
        assert abs(oracle.alpha(ce(a) ** 2) - a) < 1e-15
    s = GOLDEN["shock_distance"]
    k = 2 * math.pi / s["lambda"]
    for c, printed in zip(s["c_e"], s["sigma_over_lambda_printed"]):
        sigma = 1.0 / (s["eps"] * (s["u0"] / c) * k)
        assert round(sigma / s["lambda"]) == printed
    v = GOLDEN["viscosities"]
    for nu, tau in zip(v["nu"], v["tau"]):
        assert abs((2 * tau - 1) / 6 - nu) < 1e-15


# ---------------------------------------------------------------- ABI ---
@pytest.mark.parametrize("args", [(2, 5, 0.8, 0.2), (5, 2, 0.8, 0.2), (5, 5, 0.5, 0.2),
                                  (5, 5, float("nan"), 0.2), (5, 5, 0.8, 0.0), (5, 5, 0.8, -0.1),
                                  (5, 5, 0.8, float("inf"))])
def test_oracle_rejects_invalid_arguments(args):
    with pytest.raises(oracle.lbmref.OracleError) as ei:
        oracle.Oracle(*args)
    assert ei.value.status == -1


def test_oracle_step_before_init_is_state_error():
    o = oracle.Oracle(4, 4, 0.8, 0.2)
    with pytest.raises(oracle.lbmref.OracleError) as ei:
        o.step(1)
    assert ei.value.status == -4


def test_oracle_nonfinite_totals_detected():
    o = oracle.Oracle(4, 4, 0.8, 0.2)
    rho = np.ones((4, 4))
    rho[1, 2] = np.nan
    o.init(rho)
    with pytest.raises(oracle.lbmref.OracleError) as ei:
        o.moments()
    assert ei.value.status == -5
