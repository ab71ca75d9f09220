"""Seeded synthetic workloads (host FP64 fields), shared by tests and bench.

These generators hold none of the method's arithmetic: they only build the
initial density and velocity fields that both the GPU library and the CPU
oracle receive through init. The shapes follow the paper's plane sound
waves (Sec. 4: a progressive wave has delta rho / rho0 = u / c_e) and shear
waves; the paper uses no public dataset.
"""
import numpy as np

# c^2 sweep of the plain-kernel workload: c_e = 0.2 ... 0.9 (the paper's
# waves (1) and (2) are the end points, Sec. 4).
C2_SWEEP = (0.04, 0.2, 1.0 / 3.0, 0.5, 0.81)
# the altered-equilibrium model needs c^2 < 3/5 (positive rest population)
C2_SWEEP_EQ = (0.04, 0.2, 1.0 / 3.0, 0.5, 0.56)


def grid(nx, ny):
    y, x = np.mgrid[0:ny, 0:nx]
    return x.astype(np.float64), y.astype(np.float64)


def c1_fields(n=64, amp=1e-3):
    """64 x 64 parity case: rho = 1 + 1e-3 sin(2 pi x / 64), u = 0."""
    x, _ = grid(n, n)
    return 1.0 + amp * np.sin(2 * np.pi * x / n), None, None


def plane_wave_fields(nx, ny, c2, amp=1e-3, noise=1e-4, seed=0):
    """Right-going plane sound wave of relative amplitude `amp` plus seeded
    uniform density noise in [-noise, noise]:
        rho = 1 + amp sin(2 pi x / nx) + xi,  u_x = sqrt(c2) amp sin(2 pi x / nx),  u_y = 0."""
    x, _ = grid(nx, ny)
    s = np.sin(2 * np.pi * x / nx)
    rng = np.random.default_rng(seed)
    xi = rng.uniform(-noise, noise, size=(ny, nx)) if noise > 0 else 0.0
    return 1.0 + amp * s + xi, np.sqrt(c2) * amp * s, None


def simple_wave_fields(nx, ny, c2, u0):
    """A right-going simple wave of finite amplitude (the paper's nonlinear
    progressive waves, Sec. 4): u_x = u0 sin(2 pi x / nx) and rho =
    exp(u_x / c), the relation that holds along a right-going simple wave of
    a gas with p = c^2 rho (its Riemann invariant u - c ln rho is zero), so
    that no left-going wave is excited at any order."""
    x, _ = grid(nx, ny)
    u = u0 * np.sin(2 * np.pi * x / nx)
    return np.exp(u / np.sqrt(c2)), u, None


def shear_wave_fields(nx, ny, amp=0.01):
    """Shear wave u_x = amp sin(2 pi y / ny), rho = 1 (x-invariant)."""
    _, y = grid(nx, ny)
    return None, amp * np.sin(2 * np.pi * y / ny), None


def gaussian_pulse_fields(nx, ny, amp, sigma=None):
    """Centred Gaussian density pulse rho = 1 + amp exp(-r^2 / (2 sigma^2)), u = 0."""
    sigma = sigma if sigma is not None else min(nx, ny) / 16.0
    x, y = grid(nx, ny)
    r2 = (x - nx / 2.0) ** 2 + (y - ny / 2.0) ** 2
    return 1.0 + amp * np.exp(-r2 / (2.0 * sigma * sigma)), None, None


def lens_c2_field(nx, ny, c2, depth=0.5, noise=0.0, seed=0):
    """A c^2 field shaped like an acoustic lens (the paper's example of a
    pre-determined variation, Sec. 5): c^2 (1 - depth exp(-r^2 / (2 sigma^2)))
    around the centre, sigma = min(nx, ny) / 6, times a seeded factor
    1 + U[-noise, noise] per site (so that every site differs)."""
    x, y = grid(nx, ny)
    sigma = min(nx, ny) / 6.0
    r2 = (x - nx / 2.0) ** 2 + (y - ny / 2.0) ** 2
    f = c2 * (1.0 - depth * np.exp(-r2 / (2.0 * sigma * sigma)))
    if noise > 0:
        f = f * (1.0 + np.random.default_rng(seed).uniform(-noise, noise, size=(ny, nx)))
    return f


def batch_specs(n=256, seed=0, lo=64, hi=1024):
    """The batching workload: n independent periodic lattices with
    nx, ny ~ U{lo..hi}, tau ~ U[0.55, 1.5], c^2 ~ U[0.04, 0.6] (inside the
    linearly stable range for tau >= 0.55) and a centred Gaussian density
    pulse of amplitude ~ U[0.01, 0.1] (width min(nx, ny)/16) at rest.
    Returns a list of dicts (nx, ny, tau, c2, amp)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        out.append({"nx": int(rng.integers(lo, hi + 1)), "ny": int(rng.integers(lo, hi + 1)),
                    "tau": float(rng.uniform(0.55, 1.5)), "c2": float(rng.uniform(0.04, 0.6)),
                    "amp": float(rng.uniform(0.01, 0.1))})
    return out


def batch_fields(spec):
    """Initial fields of one lattice of batch_specs()."""
    return gaussian_pulse_fields(spec["nx"], spec["ny"], spec["amp"])
