"""Two-pass predictor-corrector time step (section 3.3), FP64 oracle.

One step from t to t + dt, following the paper's order:

pass 1 (V_c = V_0, thetadot_c = thetadot_0), pass 2 (V_c = (V_0 + V_1)/2,
thetadot_c = (thetadot_0 + thetadot_1)/2), each pass doing

  (1) predict slip u_p = u_0 + dt V_c and state theta_p = theta_0 + dt thetadot_c
  (2) tractions at t + dt: static term on the predicted slip, the current
      interval's rate V_c with weight w_{n,0} (the integral over [0, dt]),
      and the stored history with weights w_{n,j}, j >= 1 (section 3.1)
  (3) Newton solve of the momentum balance for V_p, then
      thetadot_p = 1 - theta_p V_p / Dc (aging law).

The step ends with u = u_2, V = V_2, theta = theta_2, thetadot = thetadot_2,
and the rate stored in the spectral history for the interval [t, t+dt] is
(V_0 + V_1)/2, the rate that moved the slip in pass 2.

Readings (the paper is silent on them):
* loading is backslip at the plate rate V_pl: the elastic terms act on
  Delta u - V_pl t and V - V_pl, and a uniform V_pl is an exact steady state;
  an optional uniform shear-load rate adds tau_rate * t;
* the history before the first step is V = V_pl (zero in the backslip
  frame);
* theta update: ``theta_mode="paper"`` is the explicit update above (the
  paper's); ``"exp"`` integrates the aging law exactly at the fixed rate
  V_c: theta_p = Dc/V_c + (theta_0 - Dc/V_c) exp(-V_c dt / Dc), which stays
  positive where the explicit update is unstable (V dt / Dc > 2).
* a failed step (normal traction not compressive, state not positive, or a
  Newton solve that does not converge) raises ``OracleStepError`` and leaves
  the state at the start of the step (section 3.2).
"""

from __future__ import annotations

import numpy as np

from .friction import ElementFailure, predict_state, update_elements
from .spectral import curvature, curvature_fft, odd_sign, transforms, wavenumbers
from .windows import KC_TIMES_L, KernelTable, interval_weights, midpoint_weights

ERR_NEWTON = -4
ERR_STATE = -5
ERR_OPEN = -6
FAILURE_CODES = {"newton": ERR_NEWTON, "state": ERR_STATE, "open": ERR_OPEN}


class OracleStepError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(msg)
        self.code = code


class OracleFault:
    """One periodic fault integrated by the oracle's two-pass scheme."""

    def __init__(self, N, L, mu, cs, cp, *, dt, friction, h=None, kappa=None,
                 table: KernelTable | None = None, theta_mode="paper",
                 transform="naive", max_lag=None, closure=None, rule="R1",
                 kc=(KC_TIMES_L, KC_TIMES_L)):
        """``transform``: "naive" (explicit DFT sums) or "fft" (numpy FFT);
        ``max_lag``: keep only window lags below it, which limits the run to
        max_lag steps from the state set (longer runs raise); ``closure``:
        (params_T, params_N, cut) to keep ceil(cut M_n) lags and close the
        tail with the networks of ``oracle.closure`` (bfloat16 inference);
        ``rule``: "R1" midpoint weights or "R2" exact interval integrals
        (``oracle.windows``); ``kc``: k_c L of the shear and normal windows."""
        self.N, self.L, self.mu, self.cs, self.cp, self.dt = N, L, mu, cs, cp, dt
        self._fwd, self._inv = transforms(transform)
        self.max_lag = max_lag
        self.r = (cs / cp) ** 2
        if kappa is None:
            hh = np.zeros(N) if h is None else np.asarray(h, float)
            kappa = curvature_fft(hh, L) if transform == "fft" else curvature(hh, L)
        self.kappa = np.asarray(kappa, dtype=np.float64)
        self.kabs = np.abs(wavenumbers(N, L))
        self.s = odd_sign(N)
        if rule == "R1":
            self.w = midpoint_weights(N, L, cs, cp, dt, table, max_lag=max_lag, kc=kc)
        elif rule == "R2":
            self.w = interval_weights(N, L, cs, cp, dt, max_lag=max_lag, kc=kc)
        else:
            raise ValueError("rule must be R1 or R2")
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
        # history of lags j = 1..M_n-1 (M'_n - 1 with the closure), newest
        # first, flat per mode
        M = self.w.M
        self.closure = closure
        if closure is not None:
            from .closure import kept_lags
            self.M_kept, self.closed = kept_lags(M, closure[2])
            M = self.M_kept
        self.hM = np.maximum(M - 1, 0)
        self.hoff = np.concatenate([[0], np.cumsum(self.hM)[:-1]]).astype(np.int64)
        tot = int(self.hM.sum())
        self.HT = np.zeros(tot, dtype=np.complex128)
        self.HN = np.zeros(tot, dtype=np.complex128)
        mode_of = np.repeat(np.arange(N), self.hM)
        lag = np.arange(tot) - np.repeat(self.hoff, self.hM) + 1       # j = 1..M-1
        self._hist_mode = mode_of
        self._wT_hist = self.w.wT[self.w.off[mode_of] + lag]
        self._wN_hist = self.w.wN[self.w.off[mode_of] + lag]
        self._w0T = self.w.wT[self.w.off]
        self._w0N = self.w.wN[self.w.off]
        # shift map: entry at lag j moves to lag j+1; lag 1 receives the push
        src = np.arange(tot) - 1
        first = np.zeros(tot, dtype=bool)
        first[self.hoff[self.hM > 0]] = True
        self._shift_src = np.where(first, 0, src)
        self._first = first
        self.set_state(f["slip0"], f["V0"], f["theta0"], 0.0)

    # ------------------------------------------------------------------
    def set_state(self, slip, V, theta, t):
        self.slip = np.array(slip, dtype=np.float64)
        self.V = np.where(self.free, np.asarray(V, dtype=np.float64), self.V_pl)
        self.theta = np.array(theta, dtype=np.float64)
        self.thetadot = np.where(self.free, 1.0 - self.theta * self.V / self.Dc, 0.0)
        self.t = float(t)
        self.HT[:] = 0
        self.HN[:] = 0
        self.tau_el = np.zeros(self.N)
        self.sigma_el = np.zeros(self.N)
        self.tau_static = np.zeros(self.N)
        self.sigma_static = np.zeros(self.N)
        self.nsteps = 0

    def history_sums(self):
        """S^X_n = sum_{j>=1} w^X_{n,j} H^X_n(lag j) (plus the closed tail)."""
        ST = np.bincount(self._hist_mode, weights=(self._wT_hist * self.HT).real, minlength=self.N) \
            + 1j * np.bincount(self._hist_mode, weights=(self._wT_hist * self.HT).imag, minlength=self.N)
        SN = np.bincount(self._hist_mode, weights=(self._wN_hist * self.HN).real, minlength=self.N) \
            + 1j * np.bincount(self._hist_mode, weights=(self._wN_hist * self.HN).imag, minlength=self.N)
        if self.closure is not None:
            tT, tN = self.closure_tails()
            ST = ST + tT
            SN = SN + tN
        return ST, SN

    def history_at(self, n, lag, kind):
        """Stored history value of spectral index n at lag (1..hM[n])."""
        H = self.HT if kind == 0 else self.HN
        return H[self.hoff[n] + lag - 1]

    def _closure_inputs(self, n, kind, Mk):
        from .closure import features
        H = self.HT if kind == 0 else self.HN
        lags = np.zeros(Mk, dtype=np.complex128)
        lags[1:Mk] = H[self.hoff[n]:self.hoff[n] + Mk - 1]
        Tcut = self.cs * self.kabs[n] * Mk * self.dt
        return features(lags, Mk, Tcut)

    def closure_tails(self):
        """Network tails of the closed modes n = 1..N/2, mirrored as complex
        conjugates to N - n (so the spectra stay Hermitian)."""
        from .closure import discarded_weight, forward, oldest_kept, tail_from_output
        pT, pN, _ = self.closure
        tails = [np.zeros(self.N, dtype=np.complex128), np.zeros(self.N, dtype=np.complex128)]
        modes = [n for n in range(1, self.N // 2 + 1) if self.closed[n]]
        for kind, params in ((0, pT), (1, pN)):
            if not modes:
                continue
            xs, rs = zip(*(self._closure_inputs(n, kind, int(self.M_kept[n])) for n in modes))
            y = forward(params, np.array(xs), bf16_inputs=True)
            w = self.w.wT if kind == 0 else self.w.wN
            for row, n in enumerate(modes):
                if rs[row] > 0:
                    o, Mk = self.w.off[n], int(self.M_kept[n])
                    D = discarded_weight(w[o:o + self.w.M[n]], Mk, int(self.w.M[n]))
                    t = tail_from_output(y[row], rs[row], self.cs * self.kabs[n], D,
                                         oldest_kept(xs[row], rs[row]))
                    if n == self.N - n:
                        t = t.real      # the Nyquist coefficient of a real signal is real
                    tails[kind][n] = t
                    if n != self.N - n:
                        tails[kind][self.N - n] = np.conj(t)
        return tails

    def closure_samples(self, cut=0.25):
        """Training pairs from the full (plain) history: for every mode
        n = 1..N/2 that the closure would cut and both kinds, the network
        input x, the scale r and the target output (the exact tail scaled as
        the network's output).  Returns dict(x, y, r, mode, kind, tail)."""
        from .closure import discarded_weight, features, kept_lags, target_from_tail
        if self.closure is not None:
            raise ValueError("samples need the plain (full-window) history")
        Mk, use = kept_lags(self.w.M, cut)
        xs, ys, rs, ms, ks, ts = [], [], [], [], [], []
        for kind in (0, 1):
            H = self.HT if kind == 0 else self.HN
            w = self.w.wT if kind == 0 else self.w.wN
            for n in range(1, self.N // 2 + 1):
                if not use[n]:
                    continue
                M, mk = int(self.w.M[n]), int(Mk[n])
                lags = np.zeros(M, dtype=np.complex128)
                lags[1:M] = H[self.hoff[n]:self.hoff[n] + M - 1]
                tail = np.dot(w[self.w.off[n] + mk:self.w.off[n] + M], lags[mk:M])
                x, r = features(lags, mk, self.cs * self.kabs[n] * mk * self.dt)
                if r == 0:
                    continue
                D = discarded_weight(w[self.w.off[n]:self.w.off[n] + M], mk, M)
                xs.append(x)
                ys.append(target_from_tail(tail, r, self.cs * self.kabs[n], D, lags[mk - 1]))
                rs.append(r)
                ms.append(n)
                ks.append(kind)
                ts.append(tail)
        return dict(x=np.array(xs).reshape(-1, 33), y=np.array(ys).reshape(-1, 2), r=np.array(rs),
                    mode=np.array(ms, dtype=np.int64), kind=np.array(ks, dtype=np.int64),
                    tail=np.array(ts, dtype=np.complex128))

    def tractions(self, slip_p, V_c, t_new, ST, SN):
        """Elastic tau, sigma at t_new for predicted slip and current rate V_c."""
        u = slip_p - self.V_pl * t_new
        v = V_c - self.V_pl
        U, G = self._fwd(u), self._fwd(self.kappa * u)
        Vh, GV = self._fwd(v), self._fwd(self.kappa * v)
        stat_T = -self.mu * self.kabs * (1 - self.r) * U
        stat_N = -1j * self.s * self.mu * (1 - self.r) * G
        tau_hat = stat_T - self.mu * self.kabs * (self._w0T * Vh + ST)
        sig_hat = stat_N - 1j * self.s * self.mu * (self._w0N * GV + SN)
        # static parts (the (1-r) slip terms) of the last evaluation: the FP32
        # comparison scale where static and dynamic parts cancel
        self._last_static = (stat_T, stat_N)
        return self._inv(tau_hat), self._inv(sig_hat), Vh, GV

    def _pass(self, V_c, thd_c, ST, SN):
        dt = self.dt
        t_new = self.t + dt
        slip_p = self.slip + dt * V_c
        theta_p = predict_state(self.theta, V_c, thd_c, dt, self.Dc, self.theta_mode)
        tau_el, sig_el, Vh, GV = self.tractions(slip_p, V_c, t_new, ST, SN)
        tau = self.tau_load + self.tau_rate * t_new + tau_el
        sig = self.sigma_load + sig_el
        try:
            theta_p, V_p, thd_p = update_elements(
                tau, sig, self.theta, theta_p, V_c, self.a, self.b, self.f0, self.V_ref, self.Dc,
                self.eta_rad, self.free, self.V_pl)
        except ElementFailure as e:
            raise OracleStepError(FAILURE_CODES[e.kind], str(e)) from None
        return slip_p, theta_p, V_p, thd_p, tau_el, sig_el, Vh, GV

    def step(self):
        if self.max_lag is not None and self.nsteps >= self.max_lag:
            raise ValueError("history longer than the weights kept (max_lag)")
        ST, SN = self.history_sums()
        V0, thd0 = self.V, self.thetadot
        _, _, V1, thd1, _, _, _, _ = self._pass(V0, thd0, ST, SN)
        Vc = 0.5 * (V0 + V1)
        slip2, theta2, V2, thd2, tau_el, sig_el, Vh, GV = self._pass(Vc, 0.5 * (thd0 + thd1), ST, SN)
        # push (V0 + V1)/2 as the rate of the interval [t, t + dt]
        self.HT = np.where(self._first, Vh[self._hist_mode], self.HT[self._shift_src])
        self.HN = np.where(self._first, GV[self._hist_mode], self.HN[self._shift_src])
        self.slip, self.V, self.theta, self.thetadot = slip2, V2, theta2, thd2
        self.tau_el, self.sigma_el = tau_el, sig_el
        self.tau_static = self._inv(self._last_static[0])
        self.sigma_static = self._inv(self._last_static[1])
        self.t += self.dt
        self.nsteps += 1

    def run(self, nsteps, record_every=0):
        rec = []
        for i in range(nsteps):
            self.step()
            if record_every and (i + 1) % record_every == 0:
                rec.append(dict(step=self.nsteps, slip=self.slip.copy(), V=self.V.copy(),
                                theta=self.theta.copy(), tau_el=self.tau_el.copy(),
                                sigma_el=self.sigma_el.copy()))
        return rec
