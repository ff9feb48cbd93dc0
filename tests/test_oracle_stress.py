"""Pins of the oracle's DFT, curvature and stress functional (no GPU)."""

import mpmath as mp
import numpy as np
import pytest
import scipy.signal

from oracle.bruteforce import stress_bruteforce
from oracle.kernels import kernels_mp
from oracle.spectral import curvature, curvature_fft, dft, fft_dft, fft_idft_real, idft, idft_real, wavenumbers
from oracle.stress import stress_from_history
from oracle.windows import midpoint_weights, window_steps

MU, CS, CP = 30e9, 3464.0, 6000.0
R = (CS / CP) ** 2


def test_naive_dft_matches_library_fft():
    rng = np.random.default_rng(1)
    for N in (8, 64, 96):
        f = rng.standard_normal(N) + 1j * rng.standard_normal(N)
        assert np.allclose(dft(f), np.fft.fft(f), rtol=0, atol=1e-11 * N)
        assert np.allclose(idft(dft(f)), f, rtol=0, atol=1e-13 * N)


def test_traction_multipliers_keep_real_signals_real():
    # -mu|k| is even and real, -i sgn(k) (Nyquist dropped) is odd and
    # imaginary: both map real signals to real signals.
    from oracle.spectral import odd_sign
    N, L = 64, 10e3
    f = np.random.default_rng(3).standard_normal(N)
    for mult in (-np.abs(wavenumbers(N, L)), -1j * odd_sign(N)):
        g = idft(mult * dft(f))
        assert np.abs(g.imag).max() < 1e-13 * np.abs(g.real).max()


def test_curvature_of_sinusoid_is_exact():
    N, L, A, m = 128, 10e3, 7.0, 5
    k0 = 2 * np.pi * m / L
    x = np.arange(N) * L / N
    kap = curvature(A * np.sin(k0 * x), L)
    assert np.abs(kap + A * k0 ** 2 * np.sin(k0 * x)).max() < 1e-12 * A * k0 ** 2


def _weights(N, L, dt):
    return midpoint_weights(N, L, CS, CP, dt)


def test_zero_slip_gives_zero_stress():
    N, L = 32, 10e3
    dt = 0.5 * L / N / CS
    kap = curvature(np.random.default_rng(0).standard_normal(N), L)
    tau, sig = stress_from_history(np.zeros((6, N)), dt, L, MU, CS, CP, kap, _weights(N, L, dt))
    assert np.all(tau == 0) and np.all(sig == 0)


def test_planar_fault_has_no_normal_traction_change():
    N, L = 32, 10e3
    dt = 0.5 * L / N / CS
    hist = np.cumsum(np.random.default_rng(2).random((9, N)), axis=0)
    tau, sig = stress_from_history(hist, dt, L, MU, CS, CP, np.zeros(N), _weights(N, L, dt))
    assert np.all(sig == 0) and np.abs(tau).max() > 0


def test_single_mode_static_shear():
    # Static term of the spectral shear traction: -mu(1-r)|k| u_hat.
    N, L, D, m = 64, 10e3, 0.3, 4
    x = np.arange(N) * L / N
    km = 2 * np.pi * m / L
    tau, _ = stress_from_history(D * np.cos(km * x)[None], 1e-3, L, MU, CS, CP, np.zeros(N),
                                 _weights(N, L, 1e-3))
    assert np.abs(tau + MU * (1 - R) * km * D * np.cos(km * x)).max() < 1e-12 * MU * km * D


def test_static_tractions_equal_periodic_hilbert_transforms():
    # Textbook check: the static tractions of a band-limited slip are
    # -mu(1-r) H[du/dx] (shear) and mu(1-r) H[kappa du] (normal,
    # compression positive), H the Hilbert transform (scipy's analytic signal).
    N, L = 128, 10e3
    x = np.arange(N) * L / N
    k1, k2, k3 = (2 * np.pi * m / L for m in (1, 3, 7))
    du = 1.0 + 0.4 * np.cos(k1 * x) + 0.2 * np.sin(k2 * x)
    ddu = -0.4 * k1 * np.sin(k1 * x) + 0.2 * k2 * np.cos(k2 * x)
    h = 20.0 * np.sin(k3 * x)
    kap = -20.0 * k3 ** 2 * np.sin(k3 * x)
    tau, sig = stress_from_history(du[None], 1e-3, L, MU, CS, CP, kap, _weights(N, L, 1e-3))
    H = lambda f: np.imag(scipy.signal.hilbert(f))  # noqa: E731
    assert np.abs(tau - (-MU * (1 - R) * H(ddu))).max() < 1e-10 * np.abs(tau).max()
    assert np.abs(sig - MU * (1 - R) * H(kap * du)).max() < 1e-10 * np.abs(sig).max()
    assert np.allclose(curvature(h, L), kap, atol=1e-12 * np.abs(kap).max())


def test_uniform_slip_on_restraining_bend_compresses():
    # Uniform slip D on h = A sin(k0 x): sigma = mu(1-r) D A k0^2 cos(k0 x);
    # at x = 0 (positive slope, restraining side) the fault is compressed.
    N, L, A, D, m = 64, 10e3, 15.0, 2.0, 3
    x = np.arange(N) * L / N
    k0 = 2 * np.pi * m / L
    kap = curvature(A * np.sin(k0 * x), L)
    _, sig = stress_from_history(np.full((1, N), D), 1e-3, L, MU, CS, CP, kap, _weights(N, L, 1e-3))
    ref = MU * (1 - R) * D * A * k0 ** 2 * np.cos(k0 * x)
    assert np.abs(sig - ref).max() < 1e-12 * np.abs(ref).max()
    assert sig[0] > 0


@pytest.mark.parametrize("f", [0.6, 0.3])
def test_static_scaling_law(f):
    # Section 5: (1/(f du)) d(du)/dx = -kappa.  If the curvature is chosen as
    # kappa = -(du'/du)/f then the static shear traction equals f times the
    # static (compression-positive) normal traction at every element.
    N, L = 128, 10e3
    x = np.arange(N) * L / N
    k = wavenumbers(N, L)
    du = 1.5 + np.cos(2 * np.pi * x / L) + 0.3 * np.sin(6 * np.pi * x / L)
    ddu = np.real(idft(1j * k * dft(du)))
    kap = -ddu / (f * du)
    tau, sig = stress_from_history(du[None], 1e-3, L, MU, CS, CP, kap, _weights(N, L, 1e-3))
    assert np.abs(tau - f * sig).max() < 1e-12 * np.abs(tau).max()


def test_long_time_static_stiffness_limit():
    # After all motion stops and a full window has passed, the dynamic sums
    # vanish and the tractions equal the static terms exactly.
    N, L = 32, 10e3
    dt = 0.5 * L / N / CS
    w = _weights(N, L, dt)
    Mmax = int(w.M.max())
    rng = np.random.default_rng(5)
    moving = np.cumsum(rng.random((20, N)), axis=0)
    hist = np.vstack([moving, np.repeat(moving[-1:], Mmax, axis=0)])
    kap = curvature(rng.standard_normal(N), L)
    tau, sig = stress_from_history(hist, dt, L, MU, CS, CP, kap, w)
    tau_s, sig_s = stress_from_history(hist[-1:], dt, L, MU, CS, CP, kap, w)
    assert np.array_equal(tau, tau_s) and np.array_equal(sig, sig_s)
    # one step earlier the oldest moving interval is still inside the window
    tau1, _ = stress_from_history(hist[:-1], dt, L, MU, CS, CP, kap, w)
    assert np.abs(tau1 - tau_s).max() > 0


def test_constant_rate_converges_to_continuous_solution_second_order():
    # A single mode with rate V cos(k x) switched on at t = 0 (no truncation
    # reached): the exact spectral shear traction at time t is
    # -mu|k| [ (1-r) V t + V P(c_s|k|t)/(c_s|k|) ] with P(T) the integral of C^T
    # over [0, T].  The midpoint weights converge to it as O(dt^2).
    N, L, m, V = 16, 10e3, 2, 1.0
    k = 2 * np.pi * m / L
    x = np.arange(N) * L / N
    t_end = 0.8 * L / CS
    with mp.workdps(30):
        P = float(mp.quad(lambda T: kernels_mp(T, CS, CP)[0], [0, CS * k * t_end / 4,
                                                               CS * k * t_end / 2, CS * k * t_end]))
    exact = -MU * k * ((1 - R) * V * t_end + V * P / (CS * k)) * np.cos(k * x)
    errs = []
    for nt in (25, 50, 100):
        dt = t_end / nt
        w = midpoint_weights(N, L, CS, CP, dt)
        assert window_steps(N, L, CS, dt)[m] > nt
        hist = np.outer(np.arange(nt + 1) * dt, V * np.cos(k * x))
        tau, _ = stress_from_history(hist, dt, L, MU, CS, CP, np.zeros(N), w)
        errs.append(np.abs(tau - exact).max())
    o1 = np.log2(errs[0] / errs[1])
    o2 = np.log2(errs[1] / errs[2])
    assert 1.8 < o1 < 2.2 and 1.8 < o2 < 2.2, (errs, o1, o2)


def test_long_time_shear_tends_to_static_minus_radiation_damping():
    # With a constant rate V held for a long time (window L/c_s, modes below
    # k_c), the dynamic shear term tends to +mu V/(2 c_s) because the shear
    # kernel integrates to -1/2; the radiation damping -mu V/(2 c_s) of the
    # momentum balance cancels it, leaving the static stiffness.
    N, L, m, V = 16, 10e3, 1, 1.0
    k = 2 * np.pi * m / L
    x = np.arange(N) * L / N
    dt = 0.25 * L / N / CS
    w = midpoint_weights(N, L, CS, CP, dt)
    nt = int(w.M[m])
    hist = np.outer(np.arange(nt + 1) * dt, V * np.cos(k * x))
    tau, _ = stress_from_history(hist, dt, L, MU, CS, CP, np.zeros(N), w)
    static = -MU * k * (1 - R) * V * nt * dt * np.cos(k * x)
    dyn = (tau - static)[0]
    # truncated at c_s k T_w = 2 pi: the running integral is within ~0.2 of -1/2
    assert abs(dyn / (MU * V / (2 * CS)) - 1.0) < 0.4


def test_direct_sums_in_x_match_the_spectral_functional():
    # The FFT route of the functional against its direct evaluation as
    # real-space convolutions (influence kernels built from the same
    # multipliers and weights): a check of the transforms and of the lag
    # bookkeeping, not of the kernels (those are pinned against the paper's
    # space-time kernel and closed forms in test_oracle_kernels.py).
    N, L = 16, 10e3
    dt = 0.5 * L / N / CS
    w = _weights(N, L, dt)
    rng = np.random.default_rng(11)
    hist = np.cumsum(rng.random((40, N)), axis=0) * 1e-3
    kap = curvature(rng.standard_normal(N) * 3.0, L)
    tau, sig = stress_from_history(hist, dt, L, MU, CS, CP, kap, w)
    tb, sb = stress_bruteforce(hist, dt, L, MU, CS, CP, kap, w)
    assert np.abs(tau - tb).max() < 1e-12 * np.abs(tau).max()
    assert np.abs(sig - sb).max() < 1e-12 * np.abs(sig).max()


def test_fft_transforms_match_the_explicit_sums():
    rng = np.random.default_rng(11)
    for N in (8, 64, 1024, 8192):
        f = rng.standard_normal(N) + 1j * rng.standard_normal(N)
        F = dft(f)
        assert np.max(np.abs(fft_dft(f) - F)) <= 1e-12 * np.max(np.abs(F))
        g = rng.standard_normal(N)
        G = dft(g)
        assert np.max(np.abs(fft_idft_real(G) - idft_real(G))) <= 1e-12 * np.max(np.abs(g))
        h = np.cumsum(rng.standard_normal(N))
        k = curvature(h, 1e3)
        assert np.max(np.abs(curvature_fft(h, 1e3) - k)) <= 1e-11 * np.max(np.abs(k))


def test_stress_with_fft_and_short_weights_matches_explicit_sums():
    N, L, dt, nt = 64, 10e3, 0.5 * 10e3 / 64 / CS, 9
    rng = np.random.default_rng(5)
    hist = np.cumsum(rng.standard_normal((nt + 1, N)) * 1e-3, axis=0)
    kappa = curvature(1e-3 * L * np.sin(2 * np.pi * 3 * np.arange(N) / N), L)
    w_full = midpoint_weights(N, L, CS, CP, dt)
    w_short = midpoint_weights(N, L, CS, CP, dt, max_lag=nt)
    t1, s1 = stress_from_history(hist, dt, L, MU, CS, CP, kappa, w_full)
    t2, s2 = stress_from_history(hist, dt, L, MU, CS, CP, kappa, w_short, transform="fft")
    assert np.max(np.abs(t1 - t2)) <= 1e-12 * np.max(np.abs(t1))
    assert np.max(np.abs(s1 - s2)) <= 1e-12 * np.max(np.abs(s1))
