"""Naive discrete Fourier transform and spectral curvature for the oracle.

Convention: elements at x_i = i L / N; signed frequencies
n in {-N/2+1, ..., N/2} with angular wavenumbers k_n = 2 pi n / L; forward
transform F_n = sum_i f_i exp(-i k_n x_i), inverse
f_i = (1/N) sum_n F_n exp(+i k_n x_i).  The forward sign exp(-ikx) is the one
under which both Fourier pairs of appendix B hold as printed.

``dft``/``idft`` are explicit O(N^2) sums (a matrix-vector product with the
DFT matrix built from exact integer phases).  ``fft_dft``/``fft_idft_real``
take the same transforms from numpy's FFT, a library primitive used as one
step where N is too large for the explicit sums; the tests pin them to the
explicit sums.
"""

from __future__ import annotations

import numpy as np


def signed_frequencies(N: int) -> np.ndarray:
    """n_s for array index n: n if n <= N/2 else n - N."""
    n = np.arange(N)
    return np.where(n <= N // 2, n, n - N)


def wavenumbers(N: int, L: float) -> np.ndarray:
    """k_n = 2 pi n_s / L for every array index."""
    return 2.0 * np.pi * signed_frequencies(N) / L


def odd_sign(N: int) -> np.ndarray:
    """sgn(k_n) with the Nyquist bin set to 0.

    A real signal's Nyquist coefficient is real, so an odd (imaginary)
    multiplier cannot act on it; the bin is dropped for the odd operator.
    """
    s = np.sign(signed_frequencies(N)).astype(np.float64)
    s[N // 2] = 0.0
    return s


_MATS: dict[int, np.ndarray] = {}


def _dft_matrix(N: int) -> np.ndarray:
    E = _MATS.get(N)
    if E is None:
        n = np.arange(N)
        phase = np.outer(n, n) % N             # exact integer phases
        E = np.exp(-2j * np.pi * phase / N)
        if N <= 4096:
            _MATS[N] = E
    return E


def dft(f: np.ndarray) -> np.ndarray:
    """F_n = sum_i f_i exp(-2 pi i n i / N) (naive, O(N^2))."""
    f = np.asarray(f)
    N = f.shape[-1]
    if N <= 4096:
        return f @ _dft_matrix(N).T
    out = np.empty(f.shape, dtype=np.complex128)
    n = np.arange(N)
    blk = 256
    for s in range(0, N, blk):
        rows = np.arange(s, min(N, s + blk))
        E = np.exp(-2j * np.pi * (np.outer(rows, n) % N) / N)
        out[..., rows] = f @ E.T
    return out


def idft(F: np.ndarray) -> np.ndarray:
    """f_i = (1/N) sum_n F_n exp(+2 pi i n i / N) (naive, O(N^2))."""
    F = np.asarray(F)
    return np.conj(dft(np.conj(F))) / F.shape[-1]


def idft_real(F: np.ndarray) -> np.ndarray:
    """Inverse DFT of a Hermitian spectrum: the real part of ``idft``.

    Every spectrum passed here is Hermitian by construction (real signals
    times even-real or odd-imaginary multipliers), so the imaginary part is
    rounding noise; ``tests`` check that on signals well above the noise.
    """
    return idft(F).real


def fft_dft(f: np.ndarray) -> np.ndarray:
    """The forward transform of ``dft`` by numpy's FFT (same sign and scale)."""
    return np.fft.fft(np.asarray(f), axis=-1)


def fft_idft_real(F: np.ndarray) -> np.ndarray:
    """The inverse transform of ``idft_real`` by numpy's FFT."""
    return np.fft.ifft(np.asarray(F), axis=-1).real


def transforms(kind: str):
    """(forward, inverse-real) pair: ``"naive"`` sums or ``"fft"``."""
    if kind == "naive":
        return dft, idft_real
    if kind == "fft":
        return fft_dft, fft_idft_real
    raise ValueError(kind)


def curvature(h: np.ndarray, L: float) -> np.ndarray:
    """kappa = h'' by spectral differentiation, kappa = IDFT(-k^2 DFT(h)).

    Under the small-slope approximation the curvature is the second
    derivative of the profile (section 2.2).  The Nyquist term is kept.
    """
    N = len(h)
    k = wavenumbers(N, L)
    return idft_real(-(k ** 2) * dft(h))


def curvature_fft(h: np.ndarray, L: float) -> np.ndarray:
    """``curvature`` with numpy's FFT as the transform (for large N)."""
    N = len(h)
    k = wavenumbers(N, L)
    return fft_idft_real(-(k ** 2) * fft_dft(h))
