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
