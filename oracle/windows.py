"""Truncation windows and convolution weights (section 3.1, 3.3).

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

Two options the paper discusses (section 3.1) and leaves for later:

* separate cut-off wavenumbers for the shear and the normal kernel
  (``kc=(kc_T L, kc_N L)``; the paper notes that the normal kernel converges
  more slowly).  Each kind X has its own window T_w^X and length M^X_n; the
  history kept for a mode is the longer of the two, and a kind's weights are
  zero past its own window.
* the interval rule R2 (``interval_weights``): instead of the midpoint
  value, the exact integral of the kernel over each interval, clipped at the
  window end:  w^X_{n,j} = int_{j dt}^{min((j+1) dt, T_w^X)} C^X(c_s |k_n| tau) dtau
  = [P^X(c_s|k_n| min((j+1) dt, T_w^X)) - P^X(c_s |k_n| j dt)] / (c_s |k_n|),
  with the closed-form primitives P^X of ``oracle.kernels`` (evaluated as
  the integral of C^X over the span, ``kernel_integrals_fp``).  This is the
  truncated integral of section 3.1 taken exactly on a piecewise-constant
  rate history, and the form a non-uniform step history needs.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .kernels import kernels_fp
from .spectral import signed_frequencies, wavenumbers

ETA_TRUNC = 1.0
KC_TIMES_L = 200.0


def window_time(k_abs: np.ndarray, L: float, cs: float, kc_times_L: float = KC_TIMES_L) -> np.ndarray:
    """T_w(|k|) = (eta L / c_s) * min(1, k_c / |k|), k_c = kc_times_L / (eta L)
    (200 / (eta L) in the paper)."""
    kc = kc_times_L / (ETA_TRUNC * L)
    k_abs = np.asarray(k_abs, dtype=np.float64)
    ratio = np.where(k_abs > kc, kc / np.where(k_abs > 0, k_abs, 1.0), 1.0)
    return (ETA_TRUNC * L / cs) * ratio


def window_steps(N: int, L: float, cs: float, dt: float, kc_times_L: float = KC_TIMES_L) -> np.ndarray:
    """M_n for every array index n (signed-frequency order)."""
    x = window_time(np.abs(wavenumbers(N, L)), L, cs, kc_times_L) / dt
    return np.maximum(1, np.ceil(x - 1e-9 * x)).astype(np.int64)


def _kind_windows(N, L, cs, dt, kc, max_lag):
    """(M^T, M^N, M) per array index: each kind's window length and the
    longer of the two (the history kept), capped at max_lag."""
    MT = window_steps(N, L, cs, dt, kc[0])
    MN = window_steps(N, L, cs, dt, kc[1])
    M = np.maximum(MT, MN)
    if max_lag is not None:
        M = np.minimum(M, int(max_lag))
    return MT, MN, M


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
                     table: KernelTable | None = None, max_lag: int | None = None,
                     kc=(KC_TIMES_L, KC_TIMES_L)) -> Weights:
    """w^X_{n,j} = dt * C^X(c_s |k_n| (j + 1/2) dt) for X in {T, N} (rule R1),
    zero past the kind's own window (``kc``: k_c L of the shear and the normal
    kernel).

    With ``table`` the kernel values are taken from a 30-digit table indexed
    by p = |n|(2j+1) (its delta must equal pi c_s dt / L); otherwise the
    FP64 closed forms are evaluated directly.  ``max_lag`` keeps only lags
    j < max_lag of every window (enough for a history of max_lag intervals).
    """
    MT, MN, M = _kind_windows(N, L, cs, dt, kc, max_lag)
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
    wT = np.where(j < MT[mode_of], dt * CT, 0.0)
    wN = np.where(j < MN[mode_of], dt * CN, 0.0)
    return Weights(M, off, wT, wN)


def interval_weights(N: int, L: float, cs: float, cp: float, dt: float,
                     max_lag: int | None = None, kc=(KC_TIMES_L, KC_TIMES_L)) -> Weights:
    """Rule R2: w^X_{n,j} = [P^X(c_s|k_n| min((j+1) dt, T_w^X)) - P^X(c_s|k_n| j dt)]
    / (c_s |k_n|) for j < M^X_n (zero past the kind's window and for n = 0,
    where no elastic term acts), the span integrals in FP64."""
    from .kernels import kernel_integrals_fp
    MT, MN, M = _kind_windows(N, L, cs, dt, kc, max_lag)
    off = np.concatenate([[0], np.cumsum(M)[:-1]]).astype(np.int64)
    k = np.abs(wavenumbers(N, L))
    mode_of = np.repeat(np.arange(N), M)
    j = np.arange(M.sum()) - np.repeat(off, M)
    kk = k[mode_of]
    csk = cs * kk
    out = []
    for kind, kcL in ((0, kc[0]), (1, kc[1])):
        Tcut = np.minimum(kk * L, kcL)                       # c_s |k| T_w
        Ta = np.minimum(csk * j * dt, Tcut)
        Tb = np.minimum(csk * (j + 1) * dt, Tcut)
        integral = kernel_integrals_fp(Ta, Tb, cs, cp)[kind]
        w = np.where(csk > 0, integral / np.where(csk > 0, csk, 1.0), 0.0)
        out.append(w)
    return Weights(M, off, out[0], out[1])
