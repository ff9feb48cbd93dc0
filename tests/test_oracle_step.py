"""Pins of the oracle's friction solve and time step (no GPU)."""

import numpy as np
import pytest

from oracle.friction import solve_bisection, solve_newton
from oracle.stepper import ERR_OPEN, OracleFault, OracleStepError
from sbiem_inputs import FrictionSpec, friction_fields, rough_fault

MU, CS, CP = 30e9, 3464.0, 6000.0
ETA_RAD = MU / (2 * CS)


def test_newton_matches_bisection():
    rng = np.random.default_rng(7)
    n = 4000
    sigma = rng.uniform(1e6, 1e8, n)
    a = rng.uniform(0.005, 0.03, n)
    b = rng.uniform(0.005, 0.03, n)
    theta = 10 ** rng.uniform(-6, 8, n)
    tau = sigma * rng.uniform(0.3, 0.9, n)
    V, ok = solve_newton(tau, sigma, theta, a, b, 0.6, 1e-6, 1e-3, ETA_RAD, V_guess=np.full(n, 1e-9))
    Vb = solve_bisection(tau, sigma, theta, a, b, 0.6, 1e-6, 1e-3, ETA_RAD)
    assert ok.all()
    assert np.max(np.abs(np.log(V) - np.log(Vb))) < 1e-13
    # the root satisfies the momentum balance
    res = tau - ETA_RAD * V - sigma * (0.6 + a * np.log(V / 1e-6) + b * np.log(theta * 1e-6 / 1e-3))
    assert np.max(np.abs(res) / sigma) < 1e-12


def test_newton_steady_state_returns_plate_rate():
    n = 16
    sigma = np.full(n, 50e6)
    a = np.full(n, 0.01)
    b = np.full(n, 0.015)
    V_pl = 1e-9
    theta = np.full(n, 1e-3 / V_pl)
    tau = sigma * (0.6 + (a - b) * np.log(V_pl / 1e-6)) + ETA_RAD * V_pl
    V, ok = solve_newton(tau, sigma, theta, a, b, 0.6, 1e-6, 1e-3, ETA_RAD, V_guess=np.full(n, 1e-3))
    assert ok.all() and np.max(np.abs(V / V_pl - 1)) < 1e-12


def _fault(N=32, L=10e3, overstress=0.0, alpha=3e-3, theta_mode="paper", beta=0.5):
    spec = FrictionSpec(overstress=overstress)
    fr = friction_fields(N, L, MU, CS, spec)
    dt = beta * L / N / CS
    return OracleFault(N, L, MU, CS, CP, dt=dt, friction=fr, h=rough_fault(N, L, alpha, 1),
                       theta_mode=theta_mode)


def test_uniform_plate_rate_is_exact_steady_state():
    f = _fault(overstress=0.0)
    f.run(60)
    assert np.max(np.abs(f.V / 1e-9 - 1)) < 1e-12
    assert np.max(np.abs(f.theta * 1e-9 / 1e-3 - 1)) < 1e-12
    assert np.max(np.abs(f.tau_el)) < 1e-3 and np.max(np.abs(f.sigma_el)) < 1e-3


def test_failed_step_leaves_state_unchanged():
    f = _fault(overstress=0.0)
    f.run(3)
    snap = (f.slip.copy(), f.V.copy(), f.theta.copy(), f.t)
    f.sigma_load = -f.sigma_load        # tension: the step must fail
    with pytest.raises(OracleStepError) as e:
        f.step()
    assert e.value.code == ERR_OPEN
    assert np.array_equal(f.slip, snap[0]) and np.array_equal(f.V, snap[1])
    assert np.array_equal(f.theta, snap[2]) and f.t == snap[3]


def _run_to(t_end, nt, overstress, theta_mode):
    N, L = 32, 10e3
    spec = FrictionSpec(overstress=overstress, w_nuc=1500.0)
    fr = friction_fields(N, L, MU, CS, spec)
    # start from the slip rate that balances the load at t = 0 (the elastic
    # tractions vanish at t = 0 because static and dynamic terms cancel);
    # a rate that jumps at t = 0 would cost one O(dt) first step.
    fr["V0"], ok = solve_newton(fr["tau_load"], fr["sigma_load"], fr["theta0"], fr["a"], fr["b"],
                                fr["f0"], fr["V_ref"], fr["Dc"], ETA_RAD, fr["V0"])
    assert ok.all()
    f = OracleFault(N, L, MU, CS, CP, dt=t_end / nt, friction=fr, h=rough_fault(N, L, 3e-3, 1),
                    theta_mode=theta_mode)
    f.run(nt)
    return f


@pytest.mark.parametrize("overstress,theta_mode,nts,lo,hi", [
    (6e6, "paper", (40, 80, 160), 1.95, 2.05),     # smooth, V ~ 1e-4 m/s
    (9e6, "exp", (80, 160, 320), 1.75, 2.1),       # dynamic, V up to ~4 m/s
])
def test_time_step_is_second_order(overstress, theta_mode, nts, lo, hi):
    # Section 3.3: the two-pass scheme is second-order accurate in dt.
    # Integrated to a fixed time shorter than every truncation window, dt
    # halved twice; the observed order of the slip error.
    fs = [_run_to(0.1, nt, overstress, theta_mode) for nt in nts]
    e1 = np.abs(fs[0].slip - fs[1].slip).max()
    e2 = np.abs(fs[1].slip - fs[2].slip).max()
    order = np.log2(e1 / e2)
    assert lo < order < hi, (e1, e2, order)


def test_fft_transform_and_short_weights_reproduce_the_naive_oracle():
    """The large-N configuration of the oracle (numpy FFT as the transform,
    weights kept only for the lags a short run reaches) takes the same steps
    as the explicit-DFT, full-window oracle."""
    N, L = 64, 10e3
    spec = FrictionSpec(overstress=4e6, w_nuc=800.0)
    fr = friction_fields(N, L, MU, CS, spec)
    dt = 0.5 * L / N / CS
    h = rough_fault(N, L, 5e-3, 2)
    ref = OracleFault(N, L, MU, CS, CP, dt=dt, friction=fr, h=h, theta_mode="exp")
    fast = OracleFault(N, L, MU, CS, CP, dt=dt, friction=fr, h=h, theta_mode="exp",
                       transform="fft", max_lag=12)
    for _ in range(12):
        ref.step()
        fast.step()
    for a, b in ((ref.slip, fast.slip), (ref.V, fast.V), (ref.tau_el, fast.tau_el),
                 (ref.sigma_el, fast.sigma_el)):
        assert np.max(np.abs(a - b)) <= 1e-11 * np.max(np.abs(a))
    with pytest.raises(ValueError):
        fast.step()


def _kinematic_fault(monkeypatch, N, L, beta, pulse_steps, amp, seed=3):
    """An oracle fault whose momentum balance is replaced by a prescribed
    slip rate: V(step s, x) = V_pl + amp g(s) (1 + 0.7 cos(k_1 x + phi) +
    0.3 sin(k_3 x)) with a smooth pulse g over the first ``pulse_steps``
    steps and V = V_pl exactly afterwards.  The step's other bookkeeping
    (predictor, slip update, spectral history push, window truncation) is
    the oracle's own; only the Newton root is prescribed."""
    import oracle.stepper as stepper
    spec = FrictionSpec(overstress=0.0)
    fr = friction_fields(N, L, MU, CS, spec)
    dt = beta * L / N / CS
    x = np.arange(N) * L / N
    phi = np.random.default_rng(seed).uniform(0, 2 * np.pi)
    shape = 1 + 0.7 * np.cos(2 * np.pi * x / L + phi) + 0.3 * np.sin(6 * np.pi * x / L)
    V_pl = fr["V_pl"]

    def rate_after(s):             # committed rate at the end of step s (s = 1, 2, ...)
        if s >= pulse_steps:
            return np.full(N, V_pl)
        g = np.sin(np.pi * s / pulse_steps) ** 2
        return V_pl + amp * g * shape

    f = OracleFault(N, L, MU, CS, CP, dt=dt, friction=fr, h=rough_fault(N, L, 5e-3, seed),
                    theta_mode="exp")

    def prescribed(tau, sig, theta, a, b, f0, V_ref, Dc, eta, V_guess=None):
        return rate_after(f.nsteps + 1), np.ones(N, dtype=bool)

    import oracle.friction as fm
    monkeypatch.setattr(fm, "solve_newton", prescribed)
    return f, dt


def test_stepper_history_past_the_window_equals_the_stress_functional(monkeypatch):
    """The stepper keeps a per-mode history that it shifts and truncates
    every step; the stress functional (section 3.1) instead sums the whole
    slip record directly.  Driven past the longest window several times
    (M_max = 2N = 64 lags at beta = 0.5), with motion in every retained
    interval, the stepper's tractions equal the functional's on the
    recorded slip after every step; once the motion stops and every window
    has passed, only the static stiffness terms remain, exactly."""
    from oracle.spectral import dft, idft_real, odd_sign, wavenumbers
    from oracle.stress import stress_from_history
    from oracle.windows import midpoint_weights
    N, L, beta = 32, 10e3, 0.5
    pulse = 150
    f, dt = _kinematic_fault(monkeypatch, N, L, beta, pulse, 1e-4)
    w = midpoint_weights(N, L, CS, CP, dt)
    assert int(w.M.max()) == 2 * N
    slips = [f.slip.copy()]
    worst = 0.0
    for s in range(1, pulse + 2 * N + 8):
        f.step()
        slips.append(f.slip.copy())
        if s % 7 == 0 or s in (2 * N - 1, 2 * N, 2 * N + 1, pulse, pulse + 2 * N):
            tau, sig = stress_from_history(np.array(slips), dt, L, MU, CS, CP, f.kappa, w,
                                           V_pl=f.V_pl)
            scale_t, scale_s = np.abs(tau).max(), np.abs(sig).max()
            worst = max(worst, np.abs(f.tau_el - tau).max() / scale_t,
                        np.abs(f.sigma_el - sig).max() / scale_s)
    assert worst < 1e-11, worst
    # every window has passed since the motion stopped: static terms only
    r = (CS / CP) ** 2
    u = f.slip - f.V_pl * f.t
    tau_st = idft_real(-MU * np.abs(wavenumbers(N, L)) * (1 - r) * dft(u))
    sig_st = idft_real(-1j * odd_sign(N) * MU * (1 - r) * dft(f.kappa * u))
    assert np.abs(f.tau_el - tau_st).max() <= 1e-12 * np.abs(tau_st).max()
    assert np.abs(f.sigma_el - sig_st).max() <= 1e-12 * np.abs(sig_st).max()


def test_stepper_truncation_drops_exactly_the_lags_past_the_window(monkeypatch):
    """One step before the last moving interval leaves the longest window it
    still contributes to the tractions; one step after, the tractions are the
    static ones.  A history kept one lag too long or too short fails one of
    the two."""
    from oracle.spectral import dft, idft_real, wavenumbers
    N, L, beta = 32, 10e3, 0.5
    pulse = 20
    f, dt = _kinematic_fault(monkeypatch, N, L, beta, pulse, 1e-4)
    r = (CS / CP) ** 2
    M_max = 2 * N

    def static_gap():
        u = f.slip - f.V_pl * f.t
        st = idft_real(-MU * np.abs(wavenumbers(N, L)) * (1 - r) * dft(u))
        return np.abs(f.tau_el - st).max() / np.abs(st).max()

    # the last moving interval is step pulse - 1 -> pulse (its rate (V0+V1)/2
    # is non-zero); it is at lag j = s - pulse at the end of step s and
    # contributes while j < M_max
    f.run(pulse + M_max - 1)
    assert static_gap() > 1e-9
    f.step()
    assert static_gap() < 1e-13
