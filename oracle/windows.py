"""Truncation windows and midpoint convolution weights (section 3.1, 3.3).

Window: T_w(k) = (eta L / c_s) min(1, k_c/|k|) with the truncation parameter
eta = 1 and k_c = 200/(eta L) (eq. for T_w).  k_c is read as an angular
wavenumber, the same k as in the kernels, so that the kernel argument at the
end of every window beyond k_c is c_s k T_w = 200, and modes with
|n| <= 31 keep the full window L/c_s.

Window length in steps: M_n = ceil(x - 1e-9 x) with x = T_w(|k_n|)/dt (the
small guard makes exact integers such as N/beta round down on both sides of
any comparison).

Midpoint weights (the paper states only that the convolution integrals use
a midpoint rule; the reading is): the integral over the interval of lag
[j dt, (j+1) dt] is dt * C(c_s |k_n| (j + 1/2) dt), j = 0..M_n-1.  j = 0 is the
current step (its rate is the unknown being solved for), j >= 1 are stored
history intervals.  Since c_s|k_n|(j+1/2)dt = (pi c_s dt / L) |n| (2j+1), every
kernel argument is an integer multiple p = |n|(2j+1) of delta = pi c_s dt / L.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .kernels import kernels_fp
from .spectral import signed_frequencies, wavenumbers

ETA_TRUNC = 1.0
KC_TIMES_L = 200.0


def window_time(k_abs: np.ndarray, L: float, cs: float) -> np.ndarray:
    """T_w(|k|) = (eta L / c_s) * min(1, k_c / |k|), k_c = 200 / (eta L)."""
    kc = KC_TIMES_L / (ETA_TRUNC * L)
    k_abs = np.asarray(k_abs, dtype=np.float64)
    ratio = np.where(k_abs > kc, kc / np.where(k_abs > 0, k_abs, 1.0), 1.0)
    return (ETA_TRUNC * L / cs) * ratio


def window_steps(N: int, L: float, cs: float, dt: float) -> np.ndarray:
    """M_n for every array index n (signed-frequency order)."""
    x = window_time(np.abs(wavenumbers(N, L)), L, cs) / dt
    return np.maximum(1, np.ceil(x - 1e-9 * x)).astype(np.int64)


@dataclass
class KernelTable:
    """C^T and C^N tabulated at T_p = p * delta (p = 0..len-1)."""
    delta: float
    CT: np.ndarray
    CN: np.ndarray


@dataclass
class Weights:
    """Ragged per-mode weights: mode n owns flat entries off[n]..off[n]+M[n]-1
    (lag j = 0..M[n]-1)."""
    M: np.ndarray
    off: np.ndarray
    wT: np.ndarray
    wN: np.ndarray

    def mode(self, n: int):
        s = slice(self.off[n], self.off[n] + self.M[n])
        return self.wT[s], self.wN[s]


def midpoint_weights(N: int, L: float, cs: float, cp: float, dt: float,
                     table: KernelTable | None = None, max_lag: int | None = None) -> Weights:
    """w^X_{n,j} = dt * C^X(c_s |k_n| (j + 1/2) dt) for X in {T, N}.

    With ``table`` the kernel values are taken from a 30-digit table indexed
    by p = |n|(2j+1) (its delta must equal pi c_s dt / L); otherwise the
    FP64 closed forms are evaluated directly.  ``max_lag`` keeps only lags
    j < max_lag of every window (enough for a history of max_lag intervals).
    """
    M = window_steps(N, L, cs, dt)
    if max_lag is not None:
        M = np.minimum(M, int(max_lag))
    off = np.concatenate([[0], np.cumsum(M)[:-1]]).astype(np.int64)
    nabs = np.abs(signed_frequencies(N))
    mode_of = np.repeat(np.arange(N), M)
    j = np.arange(M.sum()) - np.repeat(off, M)
    if table is not None:
        delta = np.pi * cs * dt / L
        if abs(table.delta - delta) > 1e-13 * delta:
            raise ValueError("kernel table delta does not match pi*cs*dt/L")
        p = nabs[mode_of] * (2 * j + 1)
        if p.max() >= len(table.CT):
            raise ValueError(f"kernel table too short: need p={p.max()}")
        CT, CN = table.CT[p], table.CN[p]
    else:
        k = np.abs(wavenumbers(N, L))
        T = cs * k[mode_of] * (j + 0.5) * dt
        CT, CN = kernels_fp(T, cs, cp)
    return Weights(M, off, dt * CT, dt * CN)
