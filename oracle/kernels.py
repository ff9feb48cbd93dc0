"""Mode-II kernels of the spectral BIEM, for the oracle.

All kernels are written in the dimensionless time T = c_s |k| t, with
r = c_s^2/c_p^2, q = 1/r and eta = c_p/c_s, so that c_p |k| t = eta T.

* W(x) = 1 - x J0(x) + J1(x) - psi(x), psi(x) = (pi/2) x (J1 H0 - J0 H1)
  (section 2.3, equations for W and psi; H0, H1 are Struve functions).
  W is also the tail integral of J1(t)/t from x to infinity (appendix A).
* C^T_II(T) = (T^2 + r) W(eta T) - (T^2 + 1) W(T) - r J1(eta T) + J1(T)/2
  - (T/eta) J0(eta T) + T J0(T)                       (section 2.3, eq. Ct)
* C^N_II(T) = ((q-2)^2 r/2 - r - T^2) W(eta T) + (1 + T^2 - q/2) W(T)
  + (r - (q-2)^2 r/2) J1(eta T) + (q/2 - 1) J1(T) + (T/eta) J0(eta T)
  - T J0(T)                                           (section 2.4)
* c^T_II, the rate kernel whose primitive is C^T_II (section 2.3, and the
  "primitive for shear" of appendix A).  The two printed versions disagree
  (a factor 1/2 and the power of t); the reading used is the one that is
  dimensionally consistent, in units of c_s|k|:
  c^T(T) = (1/2) [J1(T)/T + 4 T (W(eta T) - W(T)) - (4/eta) J0(eta T)
  + 3 J0(T)].  It is only used to pin C^T (dC^T/dT = c^T).

Two evaluators:

* ``*_mp``: mpmath with 30 significant digits, then rounded to FP64.  The
  closed forms cancel (terms of size ~T^(1/2) give a result of size
  ~T^(-1/2)), so FP64 evaluation loses about 1e-9 relative near T = 100;
  30 digits leave more than 20 correct.
* ``*_fp``: the same closed forms in FP64, with W evaluated so that its
  error is small in the relative sense (the form through Struve functions
  loses up to 1e-12 absolute, which the T^2 factors amplify):
    - x < 5: the Neumann series 1 - W(x) = integral_0^x J1(t)/t dt
      = J1(x) + 2 sum_{k>=1} J_{2k+1}(x) (from J1(t)/t = (J0 + J2)/2 and
      integral_0^x J_nu = 2 sum_{k>=0} J_{nu+2k+1});
    - x >= 35: W = J0 A + J1 B, which follows from the paper's W with the
      Struve functions written as H_nu = Y_nu + K_nu and the Wronskian
      J1 Y0 - J0 Y1 = 2/(pi x): A = x (pi/2 K_1 - 1), B = 1 - x pi/2 K_0.
      The large-argument series of K_nu = H_nu - Y_nu (Abramowitz & Stegun
      12.1.29 with the reflection formula of the Gamma function) give
        A ~ sum_{k>=1} (-1)^k ((2k-1)!!)^2 / ((1-2k) x^(2k-1))
          = 1/x - 3/x^3 + 45/x^5 - ...,
        B ~ sum_{k>=1} (-1)^(k+1) ((2k-1)!!)^2 / x^(2k)
          = 1/x^2 - 9/x^4 + 225/x^6 - ...,
      summed while their terms decrease (error far below 1e-16 W here);
    - in between: W(x) = W(x_a) + integral_x^{x_a} J1(t)/t dt by 8-point
      Gauss-Legendre quadrature, x_a the next of the anchors 5, 5.5, ..., 35,
      whose values come from W(35) by the same quadrature panel by panel.
  W is then within 1e-16 absolute (2e-16 relative at large x) of the
  30-digit value, and C^T, C^N within about 1e-14 for T <= 250 (pinned in
  the tests against the 30-digit evaluator).
"""

from __future__ import annotations

import os
from concurrent.futures import ProcessPoolExecutor

import mpmath as mp
import numpy as np
from scipy.special import j0 as _j0, j1 as _j1, struve as _struve

MP_DPS = 30


def _mp_consts(cs, cp):
    cs = mp.mpf(cs)
    cp = mp.mpf(cp)
    r = (cs / cp) ** 2
    return r, 1 / r, cp / cs


def W_mp(x):
    """W(x) = 1 - x J0 + J1 - psi with psi = (pi/2) x (J1 H0 - J0 H1)."""
    with mp.workdps(max(MP_DPS, mp.mp.dps)):
        x = mp.mpf(x)
        J0 = mp.besselj(0, x)
        J1 = mp.besselj(1, x)
        psi = mp.pi / 2 * x * (J1 * mp.struveh(0, x) - J0 * mp.struveh(1, x))
        return 1 - x * J0 + J1 - psi


def W_integral_mp(x):
    """W(x) by its definition: the integral of J1(t)/t from x to infinity."""
    with mp.workdps(max(MP_DPS, mp.mp.dps)):
        return mp.quadosc(lambda t: mp.besselj(1, t) / t, [mp.mpf(x), mp.inf], omega=1)


def kernels_mp(T, cs, cp):
    """(C^T_II(T), C^N_II(T)) as mpmath numbers, 30 significant digits."""
    with mp.workdps(max(MP_DPS, mp.mp.dps)):
        r, q, eta = _mp_consts(cs, cp)
        T = mp.mpf(T)
        a = eta * T
        Wa, Wb = W_mp(a), W_mp(T)
        J0a, J1a = mp.besselj(0, a), mp.besselj(1, a)
        J0b, J1b = mp.besselj(0, T), mp.besselj(1, T)
        ct = ((T ** 2 + r) * Wa - (T ** 2 + 1) * Wb - r * J1a + J1b / 2
              - (T / eta) * J0a + T * J0b)
        cn = (((q - 2) ** 2 * r / 2 - r - T ** 2) * Wa + (1 + T ** 2 - q / 2) * Wb
              + (r - (q - 2) ** 2 * r / 2) * J1a + (q / 2 - 1) * J1b
              + (T / eta) * J0a - T * J0b)
        return ct, cn


def rate_kernel_T_mp(T, cs, cp):
    """c^T_II(T) in units of c_s|k| (reading stated in the module docstring)."""
    with mp.workdps(max(MP_DPS, mp.mp.dps)):
        r, q, eta = _mp_consts(cs, cp)
        T = mp.mpf(T)
        return (mp.besselj(1, T) / T + 4 * T * (W_mp(eta * T) - W_mp(T))
                - (4 / eta) * mp.besselj(0, eta * T) + 3 * mp.besselj(0, T)) / 2


_W_SERIES, _W_ASYM = 5.0, 35.0
_GL8_X, _GL8_W = np.polynomial.legendre.leggauss(8)


def _W_asymptotic(x):
    """J0 A + J1 B with the large-argument series of A and B (see above)."""
    A = np.zeros_like(x)
    B = np.zeros_like(x)
    dfac2 = 1.0                                     # ((2k-1)!!)^2
    prev = np.full_like(x, np.inf)
    live = np.ones(x.shape, dtype=bool)
    with np.errstate(over="ignore", divide="ignore", invalid="ignore"):
        for k in range(1, 80):
            dfac2 *= float((2 * k - 1) ** 2)
            ta = (-1) ** k * dfac2 / ((1 - 2 * k) * x ** (2 * k - 1))
            tb = (-1) ** (k + 1) * dfac2 / x ** (2 * k)
            live &= np.abs(ta) < prev               # stop at the smallest term
            if not live.any():
                break
            A += np.where(live, ta, 0.0)
            B += np.where(live, tb, 0.0)
            prev = np.abs(ta)
    return _j0(x) * A + _j1(x) * B


def _W_fp(x):
    """W(x) = integral of J1(t)/t from x to infinity, FP64 (see above)."""
    from scipy.special import jv as _jv
    x = np.asarray(x, dtype=np.float64)
    out = np.empty_like(x)
    big = x >= _W_ASYM
    if big.any():
        out[big] = _W_asymptotic(x[big])
    small = x < _W_SERIES
    if small.any():
        xs = x[small]
        K = int(np.ceil((xs.max() + 40.0) / 2.0))
        acc = np.zeros_like(xs)
        for k in range(K, 0, -1):                   # smallest terms first
            acc += _jv(2 * k + 1, xs)
        out[small] = 1.0 - _j1(xs) - 2.0 * acc
    mid = ~big & ~small
    if mid.any():
        xm = x[mid]
        anchors = _W_anchors()
        ia = np.minimum(np.ceil((xm - _W_SERIES) / 0.5).astype(np.int64), len(anchors) - 1)
        xa = _W_SERIES + 0.5 * ia
        out[mid] = anchors[ia] + _j1_over_t_integral(xm, xa)
    return out


def _j1_over_t_integral(a, b):
    """integral_a^b J1(t)/t dt, one 8-point Gauss-Legendre panel (b - a <= 1/2)."""
    h = b - a
    t = a[:, None] + 0.5 * h[:, None] * (1.0 + _GL8_X[None, :])
    return 0.5 * h * ((_j1(t) / t) @ _GL8_W)


_W_ANCHORS = None


def _W_anchors():
    """W at 5, 5.5, ..., 35: W(35) from the large-argument form, then one
    quadrature panel at a time towards 5."""
    global _W_ANCHORS
    if _W_ANCHORS is None:
        xs = _W_SERIES + 0.5 * np.arange(int(round((_W_ASYM - _W_SERIES) / 0.5)) + 1)
        w = np.empty_like(xs)
        w[-1] = _W_asymptotic(np.array([_W_ASYM]))[0]
        for i in range(len(xs) - 2, -1, -1):
            w[i] = w[i + 1] + _j1_over_t_integral(xs[i:i + 1], xs[i + 1:i + 2])[0]
        _W_ANCHORS = w
    return _W_ANCHORS


def kernels_fp(T, cs, cp):
    """(C^T_II(T), C^N_II(T)) in FP64 (scipy), vectorised over T."""
    T = np.asarray(T, dtype=np.float64)
    r = (cs / cp) ** 2
    q = 1.0 / r
    eta = cp / cs
    a = eta * T
    Wa, Wb = _W_fp(a), _W_fp(T)
    J0a, J1a, J0b, J1b = _j0(a), _j1(a), _j0(T), _j1(T)
    ct = ((T ** 2 + r) * Wa - (T ** 2 + 1) * Wb - r * J1a + J1b / 2
          - (T / eta) * J0a + T * J0b)
    cn = (((q - 2) ** 2 * r / 2 - r - T ** 2) * Wa + (1 + T ** 2 - q / 2) * Wb
          + (r - (q - 2) ** 2 * r / 2) * J1a + (q / 2 - 1) * J1b
          + (T / eta) * J0a - T * J0b)
    bad = ~(np.isfinite(ct) & np.isfinite(cn))
    if np.any(bad):
        ct = np.array(ct, dtype=np.float64)
        cn = np.array(cn, dtype=np.float64)
        flat_t, flat_ct, flat_cn = T.reshape(-1), ct.reshape(-1), cn.reshape(-1)
        for i in np.flatnonzero(bad.reshape(-1)):
            a, b = kernels_mp(float(flat_t[i]), cs, cp)
            flat_ct[i] = float(a)
            flat_cn[i] = float(b)
    return ct, cn


def _table_chunk(args):
    ps, delta_str, cs, cp = args
    with mp.workdps(max(MP_DPS, mp.mp.dps)):
        delta = mp.mpf(delta_str)
        out = np.empty((len(ps), 2))
        for i, p in enumerate(ps):
            ct, cn = kernels_mp(p * delta, cs, cp)
            out[i, 0] = float(ct)
            out[i, 1] = float(cn)
        return out


def kernel_table_mp(delta, p_max, cs, cp, processes=None):
    """C^T and C^N at T_p = p * delta for p = 0..p_max, 30-digit evaluation.

    ``delta`` may be a string to carry more than FP64 digits.  Returns two
    FP64 arrays of length p_max + 1.  Work is spread over a process pool.
    """
    delta_str = delta if isinstance(delta, str) else repr(float(delta))
    ps = np.arange(p_max + 1)
    nproc = processes or min(16, os.cpu_count() or 1)
    chunks = [(ps[i::nproc * 8].tolist(), delta_str, cs, cp) for i in range(nproc * 8)]
    CT = np.empty(p_max + 1)
    CN = np.empty(p_max + 1)
    if nproc == 1:
        results = [_table_chunk(c) for c in chunks]
    else:
        with ProcessPoolExecutor(nproc) as ex:
            results = list(ex.map(_table_chunk, chunks))
    for i, res in enumerate(results):
        sel = ps[i::nproc * 8]
        CT[sel] = res[:, 0]
        CN[sel] = res[:, 1]
    return CT, CN


# ---------------------------------------------------------------------------
# Primitives P^X(T) = integral of C^X_II from 0 to T (exact interval weights)
#
# Every term of C^T and C^N has an elementary primitive in W, J0, J1 and J2
# (W' = -J1(x)/x; d/dx[x^2 J2(x)] = x^2 J1(x); d/dx[x J1(x)] = x J0(x)):
#   int_0^T x^2 W(a x) dx = T^3 W(aT)/3 + T^2 J2(aT)/(3a)
#   int_0^T W(a x) dx     = T W(aT) + (1 - J0(aT))/a
#   int_0^T J1(a x) dx    = (1 - J0(aT))/a
#   int_0^T x J0(a x) dx  = T J1(aT)/a
# (the second and fourth extend the primitives of appendix A).  Summed over
# the terms of C^T (section 2.3) and C^N (section 2.4), with a = eta or 1,
# the J0 terms of the W and J1 pieces cancel pairwise, leaving
#   P^T = T^3 [W(eta T) - W(T)]/3 + T^2 [J2(eta T)/eta - J2(T)]/3
#         + r T W(eta T) - T W(T) - (1 - J0(T))/2 - r T J1(eta T) + T J1(T)
#   P^N = A T W(eta T) + B T W(T) - T^3 [W(eta T) - W(T)]/3
#         - T^2 [J2(eta T)/eta - J2(T)]/3 + r T J1(eta T) - T J1(T)
# with A = (q-2)^2 r/2 - r and B = 1 - q/2 (the constant coefficients of
# W(eta T) and W(T) in C^N).  The weight of a history interval [tau_a, tau_b]
# of wavenumber k is [P(c_s|k| tau_b) - P(c_s|k| tau_a)] / (c_s |k|).
# ---------------------------------------------------------------------------
def primitives_mp(T, cs, cp):
    """(P^T(T), P^N(T)) as mpmath numbers, 30 significant digits (more are
    carried internally: the terms grow like T^(3/2) and cancel)."""
    with mp.workdps(max(MP_DPS, mp.mp.dps) + 10):
        r, q, eta = _mp_consts(cs, cp)
        T = mp.mpf(T)
        a = eta * T
        Wa, Wb = W_mp(a), W_mp(T)
        J0b = mp.besselj(0, T)
        J1a, J1b = mp.besselj(1, a), mp.besselj(1, T)
        J2a, J2b = mp.besselj(2, a), mp.besselj(2, T)
        cubic = T ** 3 * (Wa - Wb) / 3 + T ** 2 * (J2a / eta - J2b) / 3
        pt = cubic + r * T * Wa - T * Wb - (1 - J0b) / 2 - r * T * J1a + T * J1b
        A = (q - 2) ** 2 * r / 2 - r
        B = 1 - q / 2
        pn = A * T * Wa + B * T * Wb - cubic + r * T * J1a - T * J1b
        return +pt, +pn


def primitives_fp(T, cs, cp):
    """(P^T(T), P^N(T)) in FP64 (scipy), vectorised over T.  The terms grow
    like T^(3/2) and cancel, so the absolute error grows to about 1e-12 near
    T = 200."""
    from scipy.special import jv as _jv
    T = np.asarray(T, dtype=np.float64)
    r = (cs / cp) ** 2
    q = 1.0 / r
    eta = cp / cs
    a = eta * T
    Wa, Wb = _W_fp(a), _W_fp(T)
    J0b, J1a, J1b = _j0(T), _j1(a), _j1(T)
    J2a, J2b = _jv(2, a), _jv(2, T)
    cubic = T ** 3 * (Wa - Wb) / 3 + T ** 2 * (J2a / eta - J2b) / 3
    pt = cubic + r * T * Wa - T * Wb - (1 - J0b) / 2 - r * T * J1a + T * J1b
    A = (q - 2) ** 2 * r / 2 - r
    B = 1 - q / 2
    pn = A * T * Wa + B * T * Wb - cubic + r * T * J1a - T * J1b
    bad = ~(np.isfinite(pt) & np.isfinite(pn))
    if np.any(bad):
        pt = np.array(pt, dtype=np.float64)
        pn = np.array(pn, dtype=np.float64)
        ft, fpt, fpn = T.reshape(-1), pt.reshape(-1), pn.reshape(-1)
        for i in np.flatnonzero(bad.reshape(-1)):
            x, y = primitives_mp(float(ft[i]), cs, cp)
            fpt[i] = float(x)
            fpn[i] = float(y)
    return pt, pn


_GL_X, _GL_W = np.polynomial.legendre.leggauss(8)


def kernel_integrals_fp(Ta, Tb, cs, cp):
    """(int_Ta^Tb C^T dT, int_Ta^Tb C^N dT) in FP64, vectorised.

    Short spans (Tb - Ta <= 16) use composite 8-point Gauss-Legendre
    quadrature of the FP64 closed forms on panels no wider than 1/2 (far
    below the kernels' oscillation period), so the result carries the FP64
    kernels' own accuracy; longer spans use the difference of the closed-form
    primitives, whose cancellation error (about T^3 times the rounding of W)
    is small against an integral over many units of T."""
    Ta = np.asarray(Ta, dtype=np.float64)
    Tb = np.asarray(Tb, dtype=np.float64)
    Ta, Tb = np.broadcast_arrays(Ta, Tb)
    out_t = np.zeros(Ta.shape)
    out_n = np.zeros(Ta.shape)
    span = Tb - Ta
    longs = span > 16.0
    if np.any(longs):
        pa = primitives_fp(Ta[longs], cs, cp)
        pb = primitives_fp(Tb[longs], cs, cp)
        out_t[longs] = pb[0] - pa[0]
        out_n[longs] = pb[1] - pa[1]
    short = (~longs) & (span != 0.0)
    if np.any(short):
        npan = np.ceil(span[short] / 0.5).astype(np.int64)
        npan = np.maximum(npan, 1)
        a, s = Ta[short], span[short]
        rt = np.zeros(a.shape)
        rn = np.zeros(a.shape)
        for m in np.unique(npan):
            sel = npan == m
            h = s[sel] / m                                   # panel width
            left = a[sel][:, None] + h[:, None] * np.arange(m)[None, :]
            x = left[:, :, None] + 0.5 * h[:, None, None] * (1.0 + _GL_X[None, None, :])
            ct, cn = kernels_fp(x, cs, cp)
            rt[sel] = 0.5 * h * np.einsum("ipq,q->i", ct, _GL_W)
            rn[sel] = 0.5 * h * np.einsum("ipq,q->i", cn, _GL_W)
        out_t[short] = rt
        out_n[short] = rn
    return out_t, out_n
