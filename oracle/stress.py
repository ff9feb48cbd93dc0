"""Spectral-time stress functional (section 3.1, equations for tau^el and
sigma_n^el with the truncated window T_w).

For a slip history Delta u^(m) at t_m = t_0 + m dt (m = 0..nt) the elastic
tractions at t_nt are, per signed wavenumber k_n,

  tau_hat_n   = -mu |k_n| [ (1-r) F[u^(nt)]_n + sum_j w^T_{n,j} F[rho^(nt-1-j)]_n ]
  sigma_hat_n = -i s_n mu [ (1-r) F[kappa u^(nt)]_n + sum_j w^N_{n,j} F[kappa rho^(nt-1-j)]_n ]

with r = c_s^2/c_p^2, rho^(l) = (Delta u^(l+1) - Delta u^(l))/dt the slip
rate over [t_l, t_{l+1}], the sums over j = 0..min(M_n, nt)-1 (midpoint
weights), and the backslip frame u = Delta u - V_pl t, rho -> rho - V_pl.

Reading of the normal traction: the printed multiplier "i" carries no
sgn(k) and no transform convention, although the kernel is odd in space.
With the forward transform exp(-ikx) fixed by appendix B the multiplier is
read as -i sgn(k_n), giving sigma compression-positive: then the static
limit satisfies the slip/curvature scaling law of section 5 exactly, and
uniform slip on a restraining bend compresses the fault.  The static normal
term printed with a slip rate is read with slip.  Radiation damping is not
part of this functional; it needs the instantaneous rate and enters the
momentum balance.
"""

from __future__ import annotations

import numpy as np

from .spectral import odd_sign, transforms, wavenumbers
from .windows import Weights


def stress_from_history(slip_hist, dt, L, mu, cs, cp, kappa, weights: Weights,
                        V_pl=0.0, t0=0.0, transform="naive", parts=False):
    """(tau^el, sigma^el) at the last snapshot of ``slip_hist`` (nt+1, N).

    ``transform``: "naive" (explicit DFT sums) or "fft" (numpy FFT).
    ``weights`` may keep only the lags below nt (``max_lag``).  With
    ``parts`` the static terms (the (1-r) slip terms) follow as two more
    arrays."""
    dft, idft_real = transforms(transform)
    slip_hist = np.asarray(slip_hist, dtype=np.float64)
    nt = slip_hist.shape[0] - 1
    N = slip_hist.shape[1]
    r = (cs / cp) ** 2
    kabs = np.abs(wavenumbers(N, L))
    s = odd_sign(N)
    t_end = t0 + nt * dt
    u = slip_hist[nt] - V_pl * t_end
    U = dft(u)
    G = dft(kappa * u)
    conv_T = np.zeros(N, dtype=np.complex128)
    conv_N = np.zeros(N, dtype=np.complex128)
    if nt > 0:
        rates = (slip_hist[1:] - slip_hist[:-1]) / dt - V_pl      # interval l
        R = dft(rates)[::-1]          # R[j] = spectrum of interval nt-1-j
        RG = dft(kappa * rates)[::-1]
        for n in range(N):
            m = min(int(weights.M[n]), nt)
            wT, wN = weights.mode(n)
            conv_T[n] = np.dot(wT[:m], R[:m, n])
            conv_N[n] = np.dot(wN[:m], RG[:m, n])
    tau_hat = -mu * kabs * ((1 - r) * U + conv_T)
    sig_hat = -1j * s * mu * ((1 - r) * G + conv_N)
    if parts:
        return (idft_real(tau_hat), idft_real(sig_hat), idft_real(-mu * kabs * (1 - r) * U),
                idft_real(-1j * s * mu * (1 - r) * G))
    return idft_real(tau_hat), idft_real(sig_hat)
