"""Time-adaptive stepping with a non-uniform slip-rate history (section 3.2),
FP64 oracle.  TEST INFRASTRUCTURE ONLY (see the package docstring).

``VariableStepFault`` takes the two-pass step of section 3.3 with any step
length.  Its history is a plain list of the committed intervals
[t_start, t_end] with the spectra of their rates (V_0 + V_1)/2 - V_pl; the
convolution of section 3.1 over a piecewise-constant rate is then exact per
interval:

  S^X_n(t_new) = sum_l H^X_n(l) w^X_n(l),
  w^X_n(l) = [P^X(c_s|k_n| min(tau_b, T_w^X)) - P^X(c_s|k_n| min(tau_a, T_w^X))] / (c_s |k_n|)

with tau_a = t_new - t_end(l) < tau_b = t_new - t_start(l) the interval's lag
span, T_w^X(k_n) the truncation window of kind X (an interval with
tau_a >= T_w^X does not contribute) and P^X the closed-form primitive of the
kernel (``oracle.kernels``; the differences are evaluated as integrals of
C^X over the span, ``kernel_integrals_fp``).  The interval of the step itself, lag span
[0, dt], has weight P^X(c_s|k_n| min(dt, T_w^X)) / (c_s|k_n|).  With a
constant dt this is the fixed-step scheme with interval weights (rule R2).

``AdaptiveController`` is the step-size control of section 3.2:

* from the state at t, one full step of dt (solution u_1) and, from the
  same state, two half steps of dt/2 (solution u_2); eps = u_1 - u_2 is the
  local error estimate (3/4 phi dt^3);
* reading of the error measure (the paper does not name the variable or the
  norm): eps = max over elements of |ln V_1 - ln V_2| and |ln theta_1 - ln
  theta_2| (slip rate and state span many decades);
* eps <= eps_0: the step is accepted with the more accurate two-half-step
  solution, and the next step is dt_0 = 0.9 (eps_0/eps)^(1/3) dt;
* eps > eps_0: the step is taken again with dt_0 = 0.9 (eps_0/eps)^(1/3) dt;
* a failed step (state not positive, Newton not converged, normal traction
  not compressive) is taken again with dt/2;
* dt never falls below dt_min = beta_min dx / c_s (beta_min = 0.25 in the
  paper); at dt_min an error above eps_0 is accepted, and a failure stops the
  run (``AdaptiveStop``);
* readings where the paper is silent: the next step grows by at most a
  factor ``growth`` (5) and never exceeds ``dt_max``; eps = 0 counts as the
  largest growth.
"""

from __future__ import annotations

import numpy as np

from .friction import ElementFailure, predict_state, update_elements
from .kernels import kernel_integrals_fp
from .spectral import curvature, curvature_fft, odd_sign, transforms, wavenumbers
from .stepper import FAILURE_CODES, OracleStepError
from .windows import ETA_TRUNC, KC_TIMES_L


class AdaptiveStop(RuntimeError):
    """A step failed at the smallest allowed step length (section 3.2)."""

    def __init__(self, code, t, msg):
        super().__init__(f"{msg} at t = {t} with dt at its minimum")
        self.code = code
        self.t = t


class VariableStepFault:
    """One periodic fault, two-pass steps of arbitrary length."""

    def __init__(self, N, L, mu, cs, cp, *, friction, h=None, kappa=None, theta_mode="paper",
                 kc=(KC_TIMES_L, KC_TIMES_L), transform="fft"):
        self.N, self.L, self.mu, self.cs, self.cp = N, L, mu, cs, cp
        self._fwd, self._inv = transforms(transform)
        self.r = (cs / cp) ** 2
        if kappa is None:
            hh = np.zeros(N) if h is None else np.asarray(h, float)
            kappa = curvature_fft(hh, L) if transform == "fft" else curvature(hh, L)
        self.kappa = np.asarray(kappa, dtype=np.float64)
        self.kabs = np.abs(wavenumbers(N, L))
        self.csk = cs * self.kabs
        self.s = odd_sign(N)
        # window of each kind in units of c_s|k| t: c_s|k| T_w = min(|k| L, k_c L)
        self.Tcut = [np.minimum(self.kabs * ETA_TRUNC * L, kcL) for kcL in kc]
        self.Tw_max = ETA_TRUNC * L / cs
        f = friction
        self.a, self.b = np.asarray(f["a"], float), np.asarray(f["b"], float)
        self.Dc, self.V_ref, self.f0 = f["Dc"], f["V_ref"], f["f0"]
        self.sigma_load = np.asarray(f["sigma_load"], float)
        self.tau_load = np.asarray(f["tau_load"], float)
        self.tau_rate = float(f.get("tau_load_rate", 0.0))
        self.V_pl = float(f["V_pl"])
        # constrained elements (optional "constrained" mask) slide at V_pl
        self.free = ~np.asarray(f.get("constrained", np.zeros(N, dtype=bool)), dtype=bool)
        self.eta_rad = mu / (2.0 * cs)
        self.theta_mode = theta_mode
        self.set_state(f["slip0"], f["V0"], f["theta0"], 0.0)

    def set_state(self, slip, V, theta, t):
        self.slip = np.array(slip, dtype=np.float64)
        self.V = np.where(self.free, np.asarray(V, dtype=np.float64), self.V_pl)
        self.theta = np.array(theta, dtype=np.float64)
        self.thetadot = np.where(self.free, 1.0 - self.theta * self.V / self.Dc, 0.0)
        self.t = float(t)
        self.intervals = []          # (t_start, t_end, F[V - V_pl], F[kappa (V - V_pl)])
        self.tau_el = np.zeros(self.N)
        self.sigma_el = np.zeros(self.N)
        self.nsteps = 0

    def save(self):
        return (self.slip.copy(), self.V.copy(), self.theta.copy(), self.thetadot.copy(), self.t,
                list(self.intervals), self.tau_el.copy(), self.sigma_el.copy(), self.nsteps)

    def restore(self, snap):
        (self.slip, self.V, self.theta, self.thetadot, self.t, self.intervals, self.tau_el,
         self.sigma_el, self.nsteps) = (snap[0].copy(), snap[1].copy(), snap[2].copy(),
                                        snap[3].copy(), snap[4], list(snap[5]), snap[6].copy(),
                                        snap[7].copy(), snap[8])

    def lag_weight(self, tau_a, tau_b):
        """(w^T, w^N) per mode of a lag span [tau_a, tau_b] (arrays broadcast
        against the modes).  The kernels depend on |k| only: the integrals
        are taken for n = 0..N/2 and mirrored to N - n."""
        h = self.N // 2 + 1
        mirror = np.where(np.arange(self.N) <= self.N // 2, np.arange(self.N),
                          self.N - np.arange(self.N))
        csk = self.csk[:h]
        safe = np.where(csk > 0, csk, 1.0)
        tau_a = np.asarray(tau_a, dtype=np.float64)
        tau_b = np.asarray(tau_b, dtype=np.float64)
        same = np.array_equal(self.Tcut[0], self.Tcut[1])
        out = []
        for kind in ((0, 1) if not same else (None,)):
            cut = self.Tcut[0 if kind is None else kind][:h]
            Ta = np.minimum(csk * tau_a, cut)
            Tb = np.minimum(csk * tau_b, cut)
            integrals = kernel_integrals_fp(Ta, Tb, self.cs, self.cp)
            for k in ((0, 1) if kind is None else (kind,)):
                w = np.where(csk > 0, integrals[k] / safe, 0.0)
                out.append(w[..., mirror])
        return out

    def history_sums(self, t_new):
        ST = np.zeros(self.N, dtype=np.complex128)
        SN = np.zeros(self.N, dtype=np.complex128)
        if not self.intervals:
            return ST, SN
        ta = np.array([t_new - iv[1] for iv in self.intervals])[:, None]
        tb = np.array([t_new - iv[0] for iv in self.intervals])[:, None]
        wT, wN = self.lag_weight(ta, tb)
        HT = np.array([iv[2] for iv in self.intervals])
        HN = np.array([iv[3] for iv in self.intervals])
        return np.sum(wT * HT, axis=0), np.sum(wN * HN, axis=0)

    def _pass(self, dt, V_c, thd_c, ST, SN, w0):
        t_new = self.t + dt
        slip_p = self.slip + dt * V_c
        theta_p = predict_state(self.theta, V_c, thd_c, dt, self.Dc, self.theta_mode)
        u = slip_p - self.V_pl * t_new
        v = V_c - self.V_pl
        U, G = self._fwd(u), self._fwd(self.kappa * u)
        Vh, GV = self._fwd(v), self._fwd(self.kappa * v)
        tau_hat = -self.mu * self.kabs * ((1 - self.r) * U + w0[0] * Vh + ST)
        sig_hat = -1j * self.s * self.mu * ((1 - self.r) * G + w0[1] * GV + SN)
        tau_el, sig_el = self._inv(tau_hat), self._inv(sig_hat)
        tau = self.tau_load + self.tau_rate * t_new + tau_el
        sig = self.sigma_load + sig_el
        try:
            theta_p, V_p, thd_p = update_elements(
                tau, sig, self.theta, theta_p, V_c, self.a, self.b, self.f0, self.V_ref, self.Dc,
                self.eta_rad, self.free, self.V_pl)
        except ElementFailure as e:
            raise OracleStepError(FAILURE_CODES[e.kind], str(e)) from None
        return slip_p, theta_p, V_p, thd_p, tau_el, sig_el, Vh, GV

    def step(self, dt):
        """One two-pass step of length dt; raises OracleStepError (state
        unchanged) on a failure."""
        dt = float(dt)
        t_new = self.t + dt
        ST, SN = self.history_sums(t_new)
        w0 = self.lag_weight(0.0, dt)
        V0, thd0 = self.V, self.thetadot
        _, _, V1, thd1, _, _, _, _ = self._pass(dt, V0, thd0, ST, SN, w0)
        slip2, theta2, V2, thd2, tau_el, sig_el, Vh, GV = self._pass(
            dt, 0.5 * (V0 + V1), 0.5 * (thd0 + thd1), ST, SN, w0)
        self.intervals.append((self.t, t_new, Vh, GV))
        # intervals whose lag exceeds every window never contribute again
        self.intervals = [iv for iv in self.intervals if t_new - iv[1] < self.Tw_max]
        self.slip, self.V, self.theta, self.thetadot = slip2, V2, theta2, thd2
        self.tau_el, self.sigma_el = tau_el, sig_el
        self.t = t_new
        self.nsteps += 1


def error_measure(V1, theta1, V2, theta2):
    """max over elements of |ln V1 - ln V2| and |ln theta1 - ln theta2|;
    equal values (constrained elements, where V may be 0) count 0."""
    def logdiff(x, y):
        with np.errstate(divide="ignore", invalid="ignore"):
            return np.where(x == y, 0.0, np.abs(np.log(x) - np.log(y)))
    return float(max(np.max(logdiff(V1, V2)), np.max(logdiff(theta1, theta2))))


class AdaptiveController:
    """Step-size control of section 3.2 around a ``VariableStepFault``."""

    def __init__(self, fault, eps0, dt_min, dt_max, growth=5.0, safety=0.9):
        if not (0 < dt_min <= dt_max) or eps0 <= 0:
            raise ValueError("need 0 < dt_min <= dt_max and eps0 > 0")
        self.f = fault
        self.eps0, self.dt_min, self.dt_max = float(eps0), float(dt_min), float(dt_max)
        self.growth, self.safety = float(growth), float(safety)
        self.log = []

    def next_dt(self, dt, eps):
        """0.9 (eps0/eps)^(1/3) dt, within [dt_min, min(dt_max, growth dt)]."""
        if eps > 0:
            d = self.safety * (self.eps0 / eps) ** (1.0 / 3.0) * dt
        else:
            d = self.growth * dt
        return min(max(d, self.dt_min), self.dt_max, self.growth * dt)

    def attempt(self, dt):
        """Full step and two half steps from the current state; returns eps
        (the state is left after the two half steps) or raises
        OracleStepError (state unchanged)."""
        f = self.f
        snap = f.save()
        try:
            f.step(dt)
            V1, th1 = f.V.copy(), f.theta.copy()
            f.restore(snap)
            f.step(0.5 * dt)
            f.step(0.5 * dt)
        except OracleStepError:
            f.restore(snap)
            raise
        return error_measure(V1, th1, f.V, f.theta), snap

    def advance(self, dt):
        """Take one accepted step starting with step length dt; returns the
        step length to try next."""
        dt = min(max(float(dt), self.dt_min), self.dt_max)
        while True:
            try:
                eps, snap = self.attempt(dt)
            except OracleStepError as e:
                if dt <= self.dt_min:
                    self.log.append(dict(t=self.f.t, dt=dt, outcome="stop", eps=None, code=e.code))
                    raise AdaptiveStop(e.code, self.f.t, str(e))
                self.log.append(dict(t=self.f.t, dt=dt, outcome="fail", eps=None, code=e.code))
                dt = max(0.5 * dt, self.dt_min)
                continue
            if eps <= self.eps0 or dt <= self.dt_min:
                self.log.append(dict(t=snap[4], dt=dt, eps=eps, code=0,
                                     outcome="accept" if eps <= self.eps0 else "floor"))
                return self.next_dt(dt, eps)
            self.log.append(dict(t=snap[4], dt=dt, outcome="reject", eps=eps, code=0))
            self.f.restore(snap)
            dt = max(self.safety * (self.eps0 / eps) ** (1.0 / 3.0) * dt, self.dt_min)

    def run(self, dt0, max_accepted, t_end=np.inf):
        dt = dt0
        n = 0
        while n < max_accepted and self.f.t < t_end:
            dt = self.advance(dt)
            n += 1
        return dt
