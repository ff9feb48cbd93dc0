"""Fault-geometry generators (seeded, synthetic).

* Rough fault: self-similar (Hurst exponent 1) random profile synthesised by
  the Fourier method of the rough-fault section ("Rough fault") of the paper.
  The printed spectral density is garbled; it is read as the two-sided
  P(k) = (2*pi)^3 * alpha^2 * |k|^-3, which reproduces the maximum slopes the
  paper prints for its alpha values (about 48*alpha at L = 10.24 km with a
  200 m minimum wavelength).
* Seamount: a Gaussian bump A*exp(-(x - x0)^2 / w^2) ("The seamount case").
* Sinusoid: A*sin(2 pi (x - x0) / lambda), the fault of the seismic-cycle
  section (its amplitude and wavelength are shown only in a figure).

Elements sit at x_i = i*L/N on the periodic domain [0, L).
"""

from __future__ import annotations

import numpy as np


def element_positions(N: int, L: float) -> np.ndarray:
    """Collocation nodes x_i = i*L/N, i = 0..N-1."""
    return np.arange(N, dtype=np.float64) * (L / N)


def rough_fault(N: int, L: float, alpha: float, seed: int,
                lambda_min: float | None = None,
                lambda_max: float | None = None) -> np.ndarray:
    """Self-similar random fault profile h(x_i) in metres.

    Fourier-series coefficients c_n (n = 1..N/2) are
    sqrt(P(k_n)/L) * (g1 + i g2)/sqrt(2) with g1, g2 standard normal draws
    from numpy's PCG64 generator seeded with ``seed`` (all g1 first, then all
    g2), P(k) = (2 pi)^3 alpha^2 |k|^-3 and k_n = 2 pi n / L.  Only
    wavelengths L/n in [lambda_min, lambda_max] are kept (defaults: 20*dx and
    L, as in the paper's rough-fault runs); c_0 = 0 and c_{N/2} is made real
    so that h is a real, zero-mean, periodic profile.
    """
    if N < 4 or N % 2:
        raise ValueError("N must be even and >= 4")
    dx = L / N
    lam_min = 20.0 * dx if lambda_min is None else float(lambda_min)
    lam_max = L if lambda_max is None else float(lambda_max)
    rng = np.random.Generator(np.random.PCG64(seed))
    n = np.arange(N // 2 + 1)
    k = 2.0 * np.pi * n / L
    g1 = rng.standard_normal(n.size)
    g2 = rng.standard_normal(n.size)
    P = np.zeros(n.size)
    wavelength = np.full(n.size, np.inf)
    wavelength[1:] = L / n[1:]
    keep = (n > 0) & (wavelength >= lam_min * (1 - 1e-12)) & (wavelength <= lam_max * (1 + 1e-12))
    P[keep] = (2.0 * np.pi) ** 3 * alpha ** 2 * k[keep] ** -3.0
    c = np.sqrt(P / L) * (g1 + 1j * g2) / np.sqrt(2.0)
    c[0] = 0.0
    c[-1] = c[-1].real
    # h(x_j) = sum_n c_n exp(i k_n x_j) over n in (-N/2, N/2] with c_{-n} = conj(c_n)
    return np.fft.irfft(c * N, N)


def seamount(N: int, L: float, A: float, w: float, x0: float | None = None) -> np.ndarray:
    """Gaussian bump h = A exp(-(x - x0)^2 / w^2), centred at L/2 by default.

    The periodic distance to the centre is used so that the profile is
    periodic on [0, L).
    """
    x = element_positions(N, L)
    c = L / 2.0 if x0 is None else float(x0)
    d = (x - c + L / 2.0) % L - L / 2.0
    return A * np.exp(-(d / w) ** 2)


def sinusoid(N: int, L: float, A: float, wavelength: float, x0: float | None = None) -> np.ndarray:
    """h = A sin(2 pi (x - x0) / wavelength), x0 = L/2 by default.

    The wavelength must divide L (a periodic profile): the curvature then
    vanishes at x0, where the fault is locally flat."""
    n = L / wavelength
    if abs(n - round(n)) > 1e-9 * max(1.0, n) or round(n) < 1:
        raise ValueError("the wavelength must divide L")
    x = element_positions(N, L)
    c = L / 2.0 if x0 is None else float(x0)
    return A * np.sin(2.0 * np.pi * (x - c) / wavelength)
