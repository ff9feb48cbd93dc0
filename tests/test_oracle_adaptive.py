"""Pins of the oracle's interval weights, separate cut-offs, variable-step
history and adaptive step-size control (sections 3.1 and 3.2; no GPU)."""

import mpmath as mp
import numpy as np
import pytest

from oracle.adaptive import AdaptiveController, AdaptiveStop, VariableStepFault, error_measure
from oracle.kernels import kernels_mp, primitives_fp, primitives_mp
from oracle.stepper import ERR_OPEN, ERR_STATE, OracleFault
from oracle.windows import interval_weights, midpoint_weights
from sbiem_inputs import FrictionSpec, friction_fields, rough_fault

MU, CS, CP = 30e9, 3464.0, 6000.0
R = (CS / CP) ** 2


# ---------------------------------------------------------------- primitives
@pytest.mark.parametrize("T", [0.3, 2.5, 11.0, 23.0])
def test_primitive_equals_quadrature_of_the_kernel(T):
    """P^X(T) (closed form) against the integral of C^X over [0, T] by
    adaptive quadrature of the section 2.3 / 2.4 closed forms."""
    with mp.workdps(30):
        pt, pn = primitives_mp(T, CS, CP)
        nodes = [mp.mpf(v) for v in np.linspace(0.0, T, 2 * int(np.ceil(T)) + 2)]
        qt = mp.quad(lambda x: kernels_mp(x, CS, CP)[0], nodes)
        qn = mp.quad(lambda x: kernels_mp(x, CS, CP)[1], nodes)
        assert abs(pt - qt) < mp.mpf("1e-25") and abs(pn - qn) < mp.mpf("1e-25")


@pytest.mark.parametrize("T", [0.7, 6.0, 150.0])
def test_primitive_derivative_is_the_kernel(T):
    with mp.workdps(40):
        ct, cn = kernels_mp(T, CS, CP)
        dt_ = mp.diff(lambda x: primitives_mp(x, CS, CP)[0], mp.mpf(T))
        dn_ = mp.diff(lambda x: primitives_mp(x, CS, CP)[1], mp.mpf(T))
        assert abs(dt_ - ct) < mp.mpf("1e-22") and abs(dn_ - cn) < mp.mpf("1e-22")


def test_primitive_small_argument_and_fp64_accuracy():
    # C(0) = -(1 - r) for both kernels: P(T) = -(1 - r) T + O(T^2)
    for kind in (0, 1):
        p = primitives_mp(1e-8, CS, CP)[kind]
        assert abs(float(p) / 1e-8 + (1 - R)) < 1e-6
    assert primitives_fp(np.array([0.0]), CS, CP)[0][0] == 0.0
    T = np.array([0.05, 1.0, 4.0, 6.2, 40.0, 120.0, 199.0])
    ft, fn = primitives_fp(T, CS, CP)
    for i, x in enumerate(T):
        mt, mn = primitives_mp(float(x), CS, CP)
        tol = 1e-13 if x < 6.5 else 1e-8
        assert abs(ft[i] - float(mt)) < tol and abs(fn[i] - float(mn)) < tol, (x, ft[i] - float(mt))


# ---------------------------------------------------------------- weights
def test_interval_weights_are_integrals_of_the_kernel():
    """R2 weights against direct quadrature of C^X(c_s|k|tau) over the
    interval (no primitive involved), including the clipped last lag."""
    N, L = 64, 10e3
    dt = 0.5 * L / N / CS
    w = interval_weights(N, L, CS, CP, dt)
    for n in (1, 5, 31, 32):
        k = 2 * np.pi * n / L
        M = int(w.M[n])
        Tw = (L / CS) * min(1.0, (200.0 / L) / k)
        for j in (0, 1, M // 2, M - 1):
            a, b = j * dt, min((j + 1) * dt, Tw)
            with mp.workdps(25):
                qt = mp.quad(lambda tau: kernels_mp(CS * k * tau, CS, CP)[0], [a, b])
                qn = mp.quad(lambda tau: kernels_mp(CS * k * tau, CS, CP)[1], [a, b])
            wt, wn = w.mode(n)
            assert abs(wt[j] - float(qt)) <= 1e-12 * abs(float(qt)) + 1e-18, (n, j)
            assert abs(wn[j] - float(qn)) <= 1e-12 * abs(float(qn)) + 1e-18, (n, j)


def test_midpoint_and_interval_rules_converge_at_second_order():
    """R1 - R2 shrinks by about 4 each time dt halves (both approximate the
    same integral; the midpoint rule's error is O(dt^2) per unit lag)."""
    N, L = 32, 10e3
    diffs = []
    for beta in (0.5, 0.25, 0.125):
        dt = beta * L / N / CS
        a = midpoint_weights(N, L, CS, CP, dt)
        b = interval_weights(N, L, CS, CP, dt)
        mode_of = np.repeat(np.arange(N), a.M)
        last = np.zeros(a.wT.size, bool)
        last[a.off + a.M - 1] = True           # the clipped last lag differs at O(dt)
        sel = (mode_of != 0) & ~last
        diffs.append(np.abs(a.wT - b.wT)[sel].max() / dt)
    r1, r2 = diffs[0] / diffs[1], diffs[1] / diffs[2]
    assert 3.0 < r1 < 4.5 and 3.5 < r2 < 4.5, (r1, r2)


def test_separate_cutoffs_lengthen_only_their_kind():
    N, L = 256, 10e3
    dt = 0.5 * L / N / CS
    base = midpoint_weights(N, L, CS, CP, dt)
    two = midpoint_weights(N, L, CS, CP, dt, kc=(200.0, 400.0))
    n = np.arange(N)
    nabs = np.minimum(n, N - n)
    longer = nabs > 400 / (2 * np.pi)                      # past the normal kernel's k_c
    mid = (nabs > 200 / (2 * np.pi)) & ~longer
    assert np.all(two.M[nabs <= 31] == base.M[nabs <= 31])
    assert np.all(two.M[mid] > base.M[mid])
    for m in np.flatnonzero(mid)[:20]:
        wt2, wn2 = two.mode(m)
        wt1, wn1 = base.mode(m)
        M1 = int(base.M[m])
        assert np.array_equal(wt2[:M1], wt1) and not np.any(wt2[M1:])
        assert np.array_equal(wn2[:M1], wn1) and np.any(wn2[M1:])


# ---------------------------------------------------------------- stepping
def _friction(N, L, overstress=0.0, w_nuc=1500.0):
    return friction_fields(N, L, MU, CS, FrictionSpec(overstress=overstress, w_nuc=w_nuc))


def test_variable_steps_of_constant_length_equal_the_interval_rule_stepper():
    """Two bookkeepings of the same scheme: the interval list of the
    variable-step oracle at a constant dt, and the fixed-step ring with R2
    weights, over 80 steps (M_max = 32) of a nucleating slow-slip phase (past every
    window; before a rupture, which would amplify their rounding
    differences)."""
    N, L = 16, 10e3
    dt = 0.5 * L / N / CS
    fr = _friction(N, L, 4e6)
    x = np.arange(N) * L / N
    h = 20.0 * np.sin(2 * np.pi * x / L) + 8.0 * np.cos(6 * np.pi * x / L)
    a = OracleFault(N, L, MU, CS, CP, dt=dt, friction=fr, h=h, theta_mode="exp",
                    transform="fft", rule="R2", kc=(200.0, 400.0))
    b = VariableStepFault(N, L, MU, CS, CP, friction=fr, h=h, theta_mode="exp",
                          kc=(200.0, 400.0))
    worst = 0.0
    for s in range(80):
        a.step()
        b.step(dt)
        if s % 10 == 9:
            for x, y in ((a.slip, b.slip), (a.V, b.V), (a.tau_el, b.tau_el),
                         (a.sigma_el, b.sigma_el)):
                worst = max(worst, np.abs(x - y).max() / np.abs(x).max())
    assert b.V.max() > 1e-6
    assert worst < 1e-11, worst


def _prescribed_rate(monkeypatch, fault, V_of_step):
    import oracle.friction as fm

    def prescribed(tau, sig, theta, a, b, f0, V_ref, Dc, eta, V_guess=None):
        return V_of_step(fault.nsteps + 1), np.ones(fault.N, dtype=bool)

    monkeypatch.setattr(fm, "solve_newton", prescribed)


def test_constant_rate_under_variable_steps_is_exact(monkeypatch):
    """A rate V(x) switched on at t = 0 and held: with exact interval weights
    the discrete convolution is exact whatever the steps, so
      tau_hat(t) = -mu|k| [(1-r) V_hat t + V_hat P^T(c_s|k| min(t, T_w)) / (c_s|k|)]
      sigma_hat(t) = -i s mu [(1-r) G_hat t + G_hat P^N(...) / (c_s|k|)]
    (the truncated integral of section 3.1 in closed form; P from 30-digit
    arithmetic), here through 60 steps of lengths spread over 50x."""
    from oracle.spectral import dft, idft_real, odd_sign, wavenumbers
    N, L = 32, 10e3
    fr = _friction(N, L)
    fr["V_pl"] = 0.0
    x = np.arange(N) * L / N
    V = 1e-3 * (1.2 + np.cos(2 * np.pi * x / L) + 0.4 * np.sin(6 * np.pi * x / L))
    fr["V0"] = V
    f = VariableStepFault(N, L, MU, CS, CP, friction=fr, h=rough_fault(N, L, 5e-3, 2),
                          theta_mode="exp")
    _prescribed_rate(monkeypatch, f, lambda s: V)
    rng = np.random.default_rng(5)
    dx = L / N
    for _ in range(60):
        f.step(dx / CS * rng.uniform(0.05, 2.5))
    t = f.t
    k = np.abs(wavenumbers(N, L))
    PT = np.zeros(N)
    PN = np.zeros(N)
    for n in range(1, N):
        Tend = min(CS * k[n] * t, min(k[n] * L, 200.0))
        pt, pn = primitives_mp(Tend, CS, CP)
        PT[n], PN[n] = float(pt) / (CS * k[n]), float(pn) / (CS * k[n])
    Vh, Gh = dft(V), dft(f.kappa * V)
    tau = idft_real(-MU * k * ((1 - R) * Vh * t + Vh * PT))
    sig = idft_real(-1j * odd_sign(N) * MU * ((1 - R) * Gh * t + Gh * PN))
    assert np.abs(f.tau_el - tau).max() <= 1e-11 * np.abs(tau).max()
    assert np.abs(f.sigma_el - sig).max() <= 1e-11 * np.abs(sig).max()


def _dynamic_state():
    """A VariableStepFault in mid-rupture (V of order 0.1 m/s): N = 16 on a
    sinusoidal 10 km fault, 60 fixed steps after a strong overstress."""
    N, L = 16, 10e3
    dt = 0.5 * L / N / CS
    fr = _friction(N, L, 9e6)
    x = np.arange(N) * L / N
    f = VariableStepFault(N, L, MU, CS, CP, friction=fr, h=20.0 * np.sin(2 * np.pi * x / L),
                          theta_mode="exp")
    for _ in range(60):
        f.step(dt)
    return f, dt


def test_step_doubling_error_scales_with_dt_cubed():
    """eps = u_1 - u_2 = (3/4) phi dt^3 (section 3.2): from one state, eps
    falls by about 8 each time dt halves."""
    f, dt = _dynamic_state()
    assert f.V.max() > 1e-2
    ctl = AdaptiveController(f, 1.0, 1e-9, 1.0)
    eps = []
    for h in (0.02 * dt, 0.01 * dt, 0.005 * dt):
        e, snap = ctl.attempt(h)
        f.restore(snap)
        eps.append(e)
    orders = np.log2(np.array(eps[:-1]) / np.array(eps[1:]))
    assert np.all((orders > 2.6) & (orders < 3.4)), (eps, orders)


def test_error_measure_and_next_step():
    V1, V2 = np.array([1e-9, 1.0]), np.array([1e-9, 1.01])
    th1, th2 = np.array([1.0, 2.0]), np.array([1.0, 2.0])
    assert error_measure(V1, th1, V2, th2) == pytest.approx(np.log(1.01), rel=1e-15)
    f, dt = _dynamic_state()
    ctl = AdaptiveController(f, 1e-3, 1e-4, 10.0)
    assert ctl.next_dt(1.0, 1e-3 / 8) == pytest.approx(0.9 * 2.0, rel=1e-14)
    assert ctl.next_dt(1.0, 0.0) == 5.0 and ctl.next_dt(4.0, 1e-12) == 10.0
    assert ctl.next_dt(1e-3, 1.0) == 1e-4


def test_controller_accepts_rejects_and_floors():
    f, dt = _dynamic_state()
    dt_min = 0.25 * (10e3 / 16) / CS
    # a loose tolerance accepts the first try and grows the step
    ctl = AdaptiveController(f, 10.0, dt_min, 1.0)
    snap = f.save()
    t0 = f.t
    nxt = ctl.advance(dt)
    assert ctl.log[-1]["outcome"] == "accept" and nxt > dt
    assert f.t == pytest.approx(t0 + dt, rel=1e-15) and f.nsteps == snap[8] + 2
    # a tolerance below what the smallest step reaches: rejections shrink dt
    # to dt_min, where the step is taken anyway
    f.restore(snap)
    ctl = AdaptiveController(f, 1e-14, dt_min, 1.0)
    ctl.advance(4 * dt)
    outs = [e["outcome"] for e in ctl.log]
    assert outs[0] == "reject" and outs[-1] == "floor" and ctl.log[-1]["dt"] == dt_min
    assert all(b["dt"] < a["dt"] for a, b in zip(ctl.log, ctl.log[1:]))


def test_failed_step_halves_dt_and_stops_at_the_floor():
    """A state update that turns negative at dt (explicit update, V dt / Dc
    > 1) but not at dt/2: the controller halves.  A fault that opens at every
    step length stops the run once dt is at its minimum."""
    N, L = 32, 10e3
    fr = _friction(N, L)
    V0 = 1.0
    fr["V0"] = np.full(N, V0)
    fr["theta0"] = np.full(N, 10 * fr["Dc"] / V0)        # thetadot = -9
    f = VariableStepFault(N, L, MU, CS, CP, friction=fr, h=rough_fault(N, L, 3e-3, 1))
    dt = 2.0e-3                                           # theta + dt thetadot < 0
    ctl = AdaptiveController(f, 10.0, 1e-5, 1.0)
    ctl.advance(dt)
    assert ctl.log[0]["outcome"] == "fail" and ctl.log[0]["code"] == ERR_STATE
    assert ctl.log[1]["dt"] == 0.5 * dt
    g = VariableStepFault(N, L, MU, CS, CP, friction=_friction(N, L), h=rough_fault(N, L, 3e-3, 1))
    g.sigma_load = -g.sigma_load
    ctl = AdaptiveController(g, 1e-3, 1e-3, 1.0)
    with pytest.raises(AdaptiveStop) as e:
        ctl.advance(8e-3)
    assert e.value.code == ERR_OPEN
    assert [x["dt"] for x in ctl.log] == [8e-3, 4e-3, 2e-3, 1e-3]
    assert ctl.log[-1]["outcome"] == "stop" and g.nsteps == 0


def test_separate_cutoffs_truncate_each_kind_at_its_own_window(monkeypatch):
    """Kinematic pulse in wavenumber 40 of an N = 128 fault, then rest (a
    uniform curvature keeps the normal kernel's input in the same mode).
    Past k_c = 200/L the shear window of mode 40 is 204 lags; the normal
    window with k_c = 400/L is the full 256.  At the end of step s the last
    moving interval (step `pulse`) is at lag s - pulse: the shear traction
    is static from lag 204 on, the normal one from lag 256 on."""
    from oracle.spectral import dft, idft_real, odd_sign, wavenumbers
    from oracle.windows import window_steps
    import oracle.stepper as stepper
    N, L = 128, 10e3
    dt = 0.5 * L / N / CS
    fr = _friction(N, L)
    x = np.arange(N) * L / N
    shape = 1e-4 * (1 + np.cos(2 * np.pi * 40 * x / L + 0.3))
    f = OracleFault(N, L, MU, CS, CP, dt=dt, friction=fr, kappa=np.full(N, 1e-5),
                    theta_mode="exp", transform="fft", kc=(200.0, 400.0))
    MT = int(window_steps(N, L, CS, dt, 200.0)[40])
    MN = int(window_steps(N, L, CS, dt, 400.0)[40])
    assert (MT, MN) == (204, 256)
    pulse = 10

    def prescribed(tau, sig, theta, a, b, f0, V_ref, Dc, eta, V_guess=None):
        s = f.nsteps + 1
        return fr["V_pl"] + (shape if s < pulse else np.zeros(N)), np.ones(N, dtype=bool)

    import oracle.friction as fm
    monkeypatch.setattr(fm, "solve_newton", prescribed)
    k = np.abs(wavenumbers(N, L))

    def gaps():
        u = f.slip - f.V_pl * f.t
        st = idft_real(-MU * k * (1 - R) * dft(u))
        ss = idft_real(-1j * odd_sign(N) * MU * (1 - R) * dft(f.kappa * u))
        return (np.abs(f.tau_el - st).max() / np.abs(st).max(),
                np.abs(f.sigma_el - ss).max() / np.abs(ss).max())

    f.run(pulse + MT - 1)
    gt, gs = gaps()
    assert gt > 1e-9 and gs > 1e-9, (gt, gs)
    f.step()
    gt, gs = gaps()
    assert gt < 1e-12 and gs > 1e-9, (gt, gs)
    f.run(MN - MT - 1)
    assert gaps()[1] > 1e-9
    f.step()
    gt, gs = gaps()
    assert gt < 1e-12 and gs < 1e-12, (gt, gs)


def test_interval_rule_converges_at_second_order_and_beats_the_midpoint_rule():
    """Weight-accuracy study (section 3.1 rules): tractions at t = 3.2 s of a
    smooth expanding slip pulse on a 10 km fault with two bends (N = 32), at
    c_s dt/dx = 0.5, 0.25, 0.125, against the interval rule at 16x finer
    steps.  The interval rule R2 (exact kernel integrals over each interval)
    converges at second order; the midpoint rule R1 is far less accurate at
    the coseismic step, where c_s |k| dt reaches pi/2 at the Nyquist mode."""
    from scipy.special import erf
    from oracle.spectral import curvature_fft
    from oracle.stress import stress_from_history
    N, L, T_end = 32, 10e3, 3.2
    x = np.arange(N) * L / N
    kap = curvature_fft(20.0 * np.sin(6 * np.pi * x / L) + 8.0 * np.cos(14 * np.pi * x / L), L)
    t0 = np.abs(x - L / 2) / 2500.0

    def stress(nt, rule):
        dt = T_end / nt
        hist = np.array([0.5 * (1 + erf((m * dt - t0 - 0.3) / 0.15)) for m in range(nt + 1)])
        w = (midpoint_weights if rule == "R1" else interval_weights)(N, L, CS, CP, dt)
        return stress_from_history(hist, dt, L, MU, CS, CP, kap, w, transform="fft")

    def rel(a, b):
        return np.abs(a - b).max() / np.abs(b).max()

    nts = (71, 142, 284)
    ref = stress(16 * nts[1], "R2")
    e2 = [rel(stress(nt, "R2")[0], ref[0]) for nt in nts]
    e1 = rel(stress(nts[0], "R1")[0], ref[0])
    print("R2 shear errors", e2, "R1 at beta 0.5", e1)
    assert 3.0 < e2[0] / e2[1] < 5.5 and 3.0 < e2[1] / e2[2] < 5.5, e2
    assert e1 > 5 * e2[0], (e1, e2)
