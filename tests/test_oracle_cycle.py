"""Pins of the oracle's constrained elements, of the slip/curvature scaling
diagnostic (section 5) and of the seismic-cycle inputs (section 6; no GPU)."""

import numpy as np
import pytest

from oracle.adaptive import VariableStepFault, error_measure
from oracle.scaling import scaled_slip_gradient, scaling_slip
from oracle.stepper import OracleFault
from sbiem_inputs import TABLE1_CYCLE, FrictionSpec, friction_fields, rough_fault, sinusoid
from sbiem_inputs.configs import workload

MU, CS, CP = 30e9, 3464.0, 6000.0


def _rupture_fields(N, L, constrained, a_out=None):
    """A nucleating rupture in the central 60 % (V_ref = V_pl, so that the
    steady friction coefficient is f0 everywhere); outside either
    constrained or velocity-strengthening with direct effect a_out."""
    spec = FrictionSpec(V_ref=1e-9, V_pl=1e-9, V_init=1e-9, overstress=9e6, w_nuc=1500.0,
                        constrained_outside=constrained)
    fr = friction_fields(N, L, MU, CS, spec)
    if a_out is not None:
        x = np.arange(N) * L / N
        outside = np.abs(x - L / 2) >= 0.3 * L
        fr["a"] = np.where(outside, a_out, fr["a"])
        # steady at V_pl = V_ref: the load is sigma f0 + eta V_pl whatever a is
        fr["tau_load"] = np.where(outside, fr["sigma_load"] * fr["f0"]
                                  + MU * fr["V_pl"] / (2 * CS), fr["tau_load"])
    return fr


def test_constrained_element_is_the_limit_of_strong_rate_strengthening():
    """A constrained element is what a velocity-strengthening element held
    at its steady state at V_pl becomes as a -> infinity: the departure of
    its slip rate is ln(V/V_pl) ~ (stress change)/(a sigma).  The rupture
    with free, strongly strengthening surroundings converges to the
    constrained one as 1/a."""
    N, L = 32, 10e3
    dt = 0.5 * (L / N) / CS
    h = rough_fault(N, L, 3e-3, 3)
    runs = {}
    for key, fr in (("held", _rupture_fields(N, L, True)),
                    (10.0, _rupture_fields(N, L, False, 10.0)),
                    (100.0, _rupture_fields(N, L, False, 100.0))):
        f = OracleFault(N, L, MU, CS, CP, dt=dt, friction=fr, h=h, theta_mode="exp",
                        transform="fft")
        f.vpeak = 0.0
        for _ in range(6):
            f.run(25)
            f.vpeak = max(f.vpeak, f.V.max())
        runs[key] = f
    held = runs["held"]
    assert held.vpeak > 0.1                         # the rupture ran (and arrested)
    assert np.all(held.V[~held.free] == 1e-9)
    e = {a: max(np.abs(runs[a].slip - held.slip).max() / np.abs(held.slip).max(),
                np.abs(runs[a].tau_el - held.tau_el).max() / np.abs(held.tau_el).max())
         for a in (10.0, 100.0)}
    assert e[100.0] < 2e-3, e
    assert 5.0 < e[10.0] / e[100.0] < 20.0, e


def test_constrained_elements_hold_v_pl_with_a_frozen_state():
    """Variable steps with V_pl = 0: constrained elements keep zero slip and
    rate and their state; thetadot is 0 there; the free ones move."""
    w = workload("sine-cycle-N4096")
    N, L = 64, 2560.0
    spec = TABLE1_CYCLE
    fr = friction_fields(N, L, w.mu, w.cs, spec)
    fr["tau_load_rate"] = 1e5                       # load fast enough to see motion
    held = fr["constrained"]
    f = VariableStepFault(N, L, w.mu, w.cs, w.cp, friction=fr,
                          h=sinusoid(N, L, 2.0, 640.0), theta_mode="exp")
    th0 = f.theta.copy()
    for dt in (1e-3, 0.5, 3.0, 0.02, 10.0, 1e-3):
        f.step(dt)
    assert np.all(f.slip[held] == 0.0) and np.all(f.V[held] == 0.0)
    assert np.all(f.theta[held] == th0[held]) and np.all(f.thetadot[held] == 0.0)
    assert np.all(f.slip[~held] > 0.0) and f.V[~held].min() > 1e-9


def test_error_measure_counts_equal_entries_as_zero():
    V1 = np.array([0.0, 1e-9, 2e-9])
    V2 = np.array([0.0, 1e-9, 1e-9])
    th = np.array([5.0, 1.0, 1.0])
    assert error_measure(V1, th, V2, th) == pytest.approx(np.log(2.0), rel=1e-15)
    assert error_measure(V1[:2], th[:2], V2[:2], th[:2]) == 0.0


# ---------------------------------------------------------------- scaling law
@pytest.mark.parametrize("f", [0.6, 0.3])
def test_scaling_diagnostic_recovers_the_curvature_at_second_order(f):
    """For the slip the scaling law predicts on a sinusoidal fault,
    du = exp(-f h'), the diagnostic equals -kappa = -h'' up to the centred
    difference's O(dx^2) error: the error falls fourfold per halving of dx."""
    L, A, lam = 10240.0, 40.0, 2560.0
    errs = []
    for N in (256, 512, 1024):
        x = np.arange(N) * L / N
        k = 2 * np.pi / lam
        slope = A * k * np.cos(k * x)
        kappa = -A * k * k * np.sin(k * x)
        r = scaled_slip_gradient(scaling_slip(slope, f, 2.0), L, f)
        errs.append(np.abs(r + kappa).max() / np.abs(kappa).max())
    assert errs[0] < 2e-3
    for e1, e2 in zip(errs, errs[1:]):
        assert 3.8 < e1 / e2 < 4.2, errs


def test_scaling_diagnostic_floor_and_linear_slip():
    N, L, f = 16, 160.0, 0.6
    u = 3.0 + 0.5 * np.arange(N)                    # linear except across the wrap
    r = scaled_slip_gradient(u, L, f, slip_floor=3.2)
    assert np.isnan(r[0]) and np.isfinite(r[1:]).all()
    # interior: exact derivative 0.5 per dx = 10 m
    assert np.allclose(r[1:-1], 0.05 / (f * u[1:-1]), rtol=1e-14, atol=0)


# ---------------------------------------------------------------- inputs
def test_sinusoid_geometry():
    N, L = 4096, 40960.0
    h = sinusoid(N, L, 80.0, 5120.0)
    assert h[N // 2] == 0.0
    assert abs(np.abs(h).max() - 80.0) < 1e-9
    # periodic: the spectrum holds only the 8th harmonic
    H = np.abs(np.fft.rfft(h))
    assert np.argmax(H) == 8 and np.delete(H, 8).max() < 1e-9 * H[8]
    with pytest.raises(ValueError):
        sinusoid(N, L, 1.0, 3000.0)


def test_cycle_workload_fields():
    """Table 1 friction on the central quarter, constrained elsewhere; the
    load is the steady traction at V_init = V_ref (sigma f0 plus radiation
    damping at V_init)."""
    w = workload("sine-cycle-N4096")
    fr = friction_fields(w.N, w.L, w.mu, w.cs, w.friction)
    free = ~fr["constrained"]
    x = np.arange(w.N) * w.dx
    assert np.array_equal(free, np.abs(x - w.L / 2) < w.L / 8)
    assert free.sum() == 1023 and w.dx == 10.0
    assert np.all(fr["a"][free] == 0.012) and np.all(fr["b"] == 0.015)
    assert fr["Dc"] == 0.01 and fr["sigma_load"][0] == 100e6 and fr["tau_load_rate"] == 0.01
    assert fr["V_pl"] == 0.0 and np.all(fr["V0"][~free] == 0.0)
    ref = 100e6 * 0.6 + 40e9 * 1e-9 / (2 * 3464.0)
    assert np.allclose(fr["tau_load"], ref, rtol=1e-15)
    assert abs(w.dt - 0.25 * 10.0 / 3464.0) < 1e-18
