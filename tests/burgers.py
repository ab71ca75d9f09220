"""Exact solution of Burgers' equation for a sine start (test helper).

u_t + u u_x = nu u_xx, u(x, 0) = u0 sin(k x). The Cole-Hopf transformation
u = -2 nu (ln phi)_x turns it into the heat equation for phi; with the
heat kernel, the solution is the weighted average
    u(x, t) = int ((x - y) / t) W dy / int W dy,
    W(y) = exp(-(x - y)^2 / (4 nu t) - (1 / (2 nu)) int_0^y u(s, 0) ds)
         = exp(R cos(k y) - (x - y)^2 / (4 nu t)) * const,  R = u0 / (2 nu k).
It is evaluated here with the weights normalised by their maximum (no
overflow or cancellation at any R), by the trapezoidal rule on a grid fine
against both scales of W (the kernel width sqrt(2 nu t) and 1 / (R k)),
over |y - x| up to u0 t (how far a characteristic travels) plus 14 kernel
widths.

This is the reference for weakly nonlinear progressive sound waves: in a
frame moving at c, the velocity of a simple wave of a gas with p = c^2 rho
obeys Burgers' equation with nonlinearity coefficient 1 (signal speed c + u)
and diffusivity equal to the sound attenuation coefficient (nu for the
paper's model, Figs. 4-5). The paper compared its waves with a numerical
Burgers solution (Sec. 4, Figs. 2-3); this closed form replaces it.
"""
import numpy as np


def velocity(u0, k, nu, t, x, chunk=256):
    """u(x, t) for an array of positions x (t > 0)."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    R = u0 / (2.0 * nu * k)
    s = np.sqrt(2.0 * nu * t)
    dy = min(s, 1.0 / (R * k + 1e-300), 2.0 * np.pi / k) / 16.0
    half = 14.0 * s + abs(u0) * t
    off = np.arange(-half, half + dy, dy)  # y - x
    out = np.empty_like(x)
    for a in range(0, len(x), chunk):
        y = x[a:a + chunk, None] + off[None, :]
        e = R * np.cos(k * y) - off[None, :] ** 2 / (4.0 * nu * t)
        w = np.exp(e - e.max(axis=1, keepdims=True))
        out[a:a + chunk] = (w * (-off[None, :] / t)).sum(1) / w.sum(1)
    return out


def harmonics(u0, k, nu, t, nmax, npts=512):
    """Amplitudes |b_n|, n = 1..nmax, of the Fourier series of u(., t)."""
    L = 2.0 * np.pi / k
    x = np.arange(npts) * (L / npts)
    c = np.fft.rfft(velocity(u0, k, nu, t, x)) * (2.0 / npts)
    return np.abs(c[1:nmax + 1])


def shock_time(u0, k):
    """Time at which the inviscid wave steepens to a shock, 1 / (k u0)
    (the distance c / (k u0) of Eq. 9)."""
    return 1.0 / (k * u0)
