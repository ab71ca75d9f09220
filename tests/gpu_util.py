"""Helpers shared by the GPU tests: seeded inputs and error measures."""
import numpy as np


def max_rel_err(f, ref):
    """max over (i, x) of |f - ref| / |ref| for full (unshifted) populations."""
    return float(np.max(np.abs(f - ref) / np.abs(ref)))


def c1_rho(nx=64, ny=64):
    x = np.arange(nx)[None, :] * np.ones((ny, 1))
    return 1.0 + 1e-3 * np.sin(2 * np.pi * x / nx)


def smooth_random_state(nx, ny, seed, amp=0.01, uamp=0.02):
    rng = np.random.default_rng(seed)
    y, x = np.mgrid[0:ny, 0:nx]
    rho = 1 + amp * np.sin(2 * np.pi * x / nx + rng.uniform(0, 6)) * np.cos(2 * np.pi * y / ny + rng.uniform(0, 6)) \
        + 0.1 * amp * rng.standard_normal((ny, nx))
    ux = uamp * np.sin(2 * np.pi * y / ny + rng.uniform(0, 6)) + 0.1 * uamp * rng.standard_normal((ny, nx))
    uy = uamp * np.cos(2 * np.pi * x / nx + rng.uniform(0, 6)) + 0.1 * uamp * rng.standard_normal((ny, nx))
    return rho, ux, uy
