"""Rate-and-state momentum balance of the time step (section 3.3, eq. momentum).

Per element, solve for the slip rate V > 0

    tau + tau_rate_t - eta_rad V
        = sigma (f0 + a ln(V / V_ref) + b ln(theta V_ref / Dc)),

where tau is the load plus the elastic shear traction, sigma the load plus
the elastic normal traction (compression positive) and eta_rad = mu/(2 c_s)
is the radiation-damping coefficient.  The printed momentum balance omits
the radiation-damping term although the text says the S-wave inertia term
carries it and that the balance is solved with Newton-Raphson; the reading
used here keeps -mu V/(2 c_s) on the shear side.  The friction "V0" of the
printed law is the reference velocity V_ref (the same symbol also names the
step-start velocity in the time step).

In x = ln V the residual g(x) = tau - eta_rad e^x - sigma (psi + a (x - ln
V_ref)), psi = f0 + b ln(theta V_ref / Dc), is strictly decreasing when
sigma > 0 and a > 0, so the root is unique.  It lies in
[x_rs - eta_rad e^{x_rs} / (sigma a), x_rs] where x_rs is the root without
radiation damping.
"""

from __future__ import annotations

import numpy as np


def _bracket(tau, sigma, theta, a, b, f0, V_ref, Dc, eta_rad):
    """Bracket [lo, hi] of the root in x = ln V.

    hi: x_rs, the root without radiation damping, is an upper bound; so is
    max(ln(tau/eta_rad), x_0) with x_0 the rate of zero friction coefficient
    (where the friction coefficient is non-negative the damping term alone
    must not exceed tau).  lo: below x_rs - eta_rad e^hi / (sigma a) the
    residual is positive.
    """
    psi = f0 + b * np.log(theta * V_ref / Dc)
    x_rs = np.log(V_ref) + (tau / sigma - psi) / a
    x_0 = np.log(V_ref) - psi / a
    with np.errstate(divide="ignore", invalid="ignore"):
        x_d = np.where(tau > 0, np.log(np.where(tau > 0, tau, 1.0) / eta_rad), np.inf)
    hi = np.minimum(np.minimum(x_rs, np.maximum(x_d, x_0)), 700.0)
    lo = x_rs - eta_rad * np.exp(hi) / (sigma * a)
    return psi, lo, hi


def residual(x, tau, sigma, psi, a, V_ref, eta_rad):
    return tau - eta_rad * np.exp(x) - sigma * (psi + a * (x - np.log(V_ref)))


def solve_newton(tau, sigma, theta, a, b, f0, V_ref, Dc, eta_rad, V_guess,
                 max_iter=100):
    """Safeguarded Newton on x = ln V.  Returns (V, converged)."""
    tau, sigma, theta, a, b = (np.asarray(v, dtype=np.float64) for v in (tau, sigma, theta, a, b))
    psi, lo, hi = _bracket(tau, sigma, theta, a, b, f0, V_ref, Dc, eta_rad)
    x = np.clip(np.log(np.asarray(V_guess, dtype=np.float64)), lo, hi)
    done = np.zeros(x.shape, dtype=bool)
    for _ in range(max_iter):
        g = residual(x, tau, sigma, psi, a, V_ref, eta_rad)
        gp = -eta_rad * np.exp(x) - sigma * a
        root = g == 0
        lo = np.where(g > 0, x, lo)
        hi = np.where(g < 0, x, hi)
        xn = x - g / gp
        outside = ~((xn > lo) & (xn < hi)) & ~root
        xn = np.where(outside, 0.5 * (lo + hi), xn)
        xn = np.where(done | root, x, xn)
        done = done | root | (np.abs(xn - x) <= 4e-16 * np.maximum(1.0, np.abs(x)))
        x = xn
        if done.all():
            break
    return np.exp(x), done


def solve_bisection(tau, sigma, theta, a, b, f0, V_ref, Dc, eta_rad, iters=200):
    """Plain bisection on the same bracket (cross-check of solve_newton)."""
    tau, sigma, theta, a, b = (np.asarray(v, dtype=np.float64) for v in (tau, sigma, theta, a, b))
    psi, lo, hi = _bracket(tau, sigma, theta, a, b, f0, V_ref, Dc, eta_rad)
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        g = residual(mid, tau, sigma, psi, a, V_ref, eta_rad)
        lo = np.where(g > 0, mid, lo)
        hi = np.where(g > 0, hi, mid)
    return np.exp(0.5 * (lo + hi))


class ElementFailure(Exception):
    """A pass's element update failed: ``kind`` is "open", "state" or
    "newton"."""

    def __init__(self, kind, message):
        super().__init__(message)
        self.kind = kind


def predict_state(theta, V_c, thd_c, dt, Dc, theta_mode):
    """State at the step's end: the paper's forward step theta + dt thetadot
    ("paper"), or the aging law integrated exactly at constant V_c ("exp")."""
    if theta_mode == "exp":
        with np.errstate(divide="ignore", invalid="ignore"):
            ss = Dc / V_c
            return ss + (theta - ss) * np.exp(-V_c * dt / Dc)
    return theta + dt * thd_c


def update_elements(tau, sig, theta, theta_p, V_c, a, b, f0, V_ref, Dc, eta_rad, free, V_pl):
    """Momentum balance and aging law of one pass at the free elements.

    Constrained elements (``free`` False; the null-slip-rate part of the
    periodic line outside the fault) keep V = V_pl, their state frozen
    (theta unchanged, thetadot = 0) and take no part in the failure checks.
    Returns (theta_p, V_p, thetadot_p); raises ElementFailure."""
    theta_p = np.where(free, theta_p, theta)
    if np.any(sig[free] <= 0):
        raise ElementFailure("open", "normal traction not compressive")
    tf = theta_p[free]
    if np.any(tf <= 0) or not np.all(np.isfinite(tf)):
        raise ElementFailure("state", "state variable not positive")
    V_p = np.full(tau.shape, float(V_pl))
    Vf, ok = solve_newton(tau[free], sig[free], tf, a[free], b[free], f0, V_ref, Dc, eta_rad,
                          V_guess=V_c[free])
    if not np.all(ok) or not np.all(np.isfinite(Vf)):
        raise ElementFailure("newton", "Newton solve did not converge")
    V_p[free] = Vf
    thd_p = np.where(free, 1.0 - theta_p * V_p / Dc, 0.0)
    return theta_p, V_p, thd_p
