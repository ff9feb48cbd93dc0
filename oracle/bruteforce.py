"""Real-space evaluation of the stress functional, tiny N only (a check of
the FFT route and the lag bookkeeping, not of the kernels: the influence
kernels below are built from the same spectral multipliers and weights).

The spectral functional of ``oracle.stress`` is a circular convolution in
space and a truncated convolution in time.  Here the same tractions are
built the slow way: real-space influence kernels

  K^X[d, l] = (1/N) sum_n exp(i k_n x_d) m^X_n w^X_{n,l}   (l < M_n)
  K^X_s[d]  = (1/N) sum_n exp(i k_n x_d) m^X_n (1 - r)

with m^T_n = -mu |k_n| and m^N_n = -i s_n mu, each mode sum written out
term by term, then

  tau_i   = sum_j K^T_s[i-j] u_j + sum_l sum_j K^T[i-j, l] rho_j^(nt-1-l)
  sigma_i = the same with kappa_j u_j and kappa_j rho_j^(nt-1-l).

No FFT, no per-mode window bookkeeping beyond the weight table itself.
O(N^2 nt) and O(N^2 M) memory: for N <= 64.
"""

from __future__ import annotations

import numpy as np

from .spectral import odd_sign, signed_frequencies, wavenumbers
from .windows import Weights


def stress_bruteforce(slip_hist, dt, L, mu, cs, cp, kappa, weights: Weights):
    slip_hist = np.asarray(slip_hist, dtype=np.float64)
    nt = slip_hist.shape[0] - 1
    N = slip_hist.shape[1]
    if N > 64:
        raise ValueError("brute force is for N <= 64")
    r = (cs / cp) ** 2
    kabs = np.abs(wavenumbers(N, L))
    s = odd_sign(N)
    ns = signed_frequencies(N)
    mT = -mu * kabs
    mN = -1j * s * mu
    lags = min(int(weights.M.max()), nt)
    KT = np.zeros((N, lags))
    KN = np.zeros((N, lags))
    KTs = np.zeros(N)
    KNs = np.zeros(N)
    for d in range(N):
        accTs = 0.0 + 0.0j
        accNs = 0.0 + 0.0j
        accT = np.zeros(lags, dtype=np.complex128)
        accN = np.zeros(lags, dtype=np.complex128)
        for n in range(N):
            e = np.exp(2j * np.pi * ((ns[n] * d) % N) / N)
            accTs += e * mT[n] * (1 - r)
            accNs += e * mN[n] * (1 - r)
            m = min(int(weights.M[n]), lags)
            wT, wN = weights.mode(n)
            accT[:m] += e * mT[n] * wT[:m]
            accN[:m] += e * mN[n] * wN[:m]
        KTs[d] = (accTs / N).real
        KNs[d] = (accNs / N).real
        KT[d] = (accT / N).real
        KN[d] = (accN / N).real
    u = slip_hist[nt]
    g = kappa * u
    rates = (slip_hist[1:] - slip_hist[:-1]) / dt
    tau = np.zeros(N)
    sig = np.zeros(N)
    for i in range(N):
        for j in range(N):
            d = (i - j) % N
            tau[i] += KTs[d] * u[j]
            sig[i] += KNs[d] * g[j]
            for l in range(lags):
                rho = rates[nt - 1 - l, j]
                tau[i] += KT[d, l] * rho
                sig[i] += KN[d, l] * kappa[j] * rho
    return tau, sig
