"""Pins of the oracle's kernel functions against what the paper and the
mathematics fix (no GPU)."""

import mpmath as mp
import numpy as np
import pytest
from scipy.integrate import quad
from scipy.special import j0, j1

from oracle.kernels import (MP_DPS, W_integral_mp, W_mp, kernels_fp, kernels_mp,
                            rate_kernel_T_mp)

CS, CP = 3464.0, 6000.0
R = (CS / CP) ** 2
Q = 1 / R
ETA = CP / CS


def test_static_dynamic_cancellation_at_t0():
    # Sections 2.3/2.4: both kernels start at -(1 - c_s^2/c_p^2) so the static
    # and dynamic terms cancel at t = 0.
    for T in (0, mp.mpf("1e-20")):
        ct, cn = kernels_mp(T, CS, CP)
        assert abs(float(ct) + (1 - R)) < 1e-15
        assert abs(float(cn) + (1 - R)) < 1e-15


@pytest.mark.parametrize("T", [0.5, 3.0, 20.0, 120.0])
def test_shear_kernel_is_primitive_of_rate_kernel(T):
    # Section 2.3: C^T_II is the time primitive of the Geubelle-Rice rate kernel.
    with mp.workdps(MP_DPS):
        d = mp.diff(lambda x: kernels_mp(x, CS, CP)[0], mp.mpf(T))
        c = rate_kernel_T_mp(T, CS, CP)
        assert abs(d - c) < mp.mpf("1e-20")


@pytest.mark.parametrize("x", [0.3, 2.0, 17.0, 60.0])
def test_W_closed_form_matches_integral_definition(x):
    # Appendix A: W(x) is the integral of J1(t)/t from x to infinity.
    with mp.workdps(MP_DPS):
        assert abs(W_mp(x) - W_integral_mp(x)) < mp.mpf("1e-18")


def _A(z, W):
    return z * j0(z) + j1(z) + 1 + z ** 2 - (1 + z ** 2) * W


def _B(z, W):
    return 1 + j1(z) - W


@pytest.mark.parametrize("T", [0.3, 2.0, 9.0, 40.0, 150.0])
def test_normal_kernel_matches_appendix_B_rebuild(T):
    # Appendix B: the normal-traction kernel assembled from the two Fourier
    # pairs, the Lame relations lambda^2/mu^2 = (q-2)^2, lambda+2mu = mu q,
    # P-wave (argument eta T) and S-wave (argument T) parts, minus the static
    # part (1 - r).  Evaluated here in mpmath from scratch.
    with mp.workdps(MP_DPS):
        T = mp.mpf(T)

        def blocks(z):
            J0, J1 = mp.besselj(0, z), mp.besselj(1, z)
            W = 1 - z * J0 + J1 - mp.pi / 2 * z * (J1 * mp.struveh(0, z) - J0 * mp.struveh(1, z))
            A = z * J0 + J1 + 1 + z ** 2 - (1 + z ** 2) * W
            B = 1 + J1 - W
            return A, B

        r = (mp.mpf(CS) / CP) ** 2
        q = 1 / r
        Ap, Bp = blocks(mp.mpf(CP) / CS * T)
        As, Bs = blocks(T)
        rebuild = r * Ap - r / 2 * (q - 2) ** 2 * Bp - As + q / 2 * Bs - (1 - r)
        cn = kernels_mp(T, CS, CP)[1]
        assert abs(rebuild - cn) < mp.mpf("1e-22")


@pytest.mark.parametrize("k", [0.7, 3.0, 11.0])
def test_fourier_pair_1_fixes_forward_sign(k):
    # Appendix B, first pair (b = 1): F[rect(x/2)/(x sqrt(1-x^2))](k)
    # = -i pi (1 + J1(k) - W(k)) with F[f](k) = int f exp(-ikx) dx.
    # The function is odd, so F = -2i int_0^1 f sin(kx) dx.
    v = quad(lambda x: np.sin(k * x) / (x * np.sqrt(1 - x * x)), 0, 1, limit=400)[0]
    W = float(W_mp(k))
    assert abs(-2 * v - (-np.pi * _B(k, W))) < 1e-9


@pytest.mark.parametrize("k", [0.7, 3.0, 11.0])
def test_fourier_pair_2_fixes_forward_sign(k):
    # Appendix B, second pair (b = 1), Hadamard finite part at x = 0:
    # F[sqrt(1-x^2)/x^3 rect(x/2)](k) = (i pi / 2) A(k).
    g = lambda x: np.sin(k * x) * np.sqrt(1 - x * x) / x  # noqa: E731
    fp = quad(lambda x: (g(x) - k) / x ** 2, 0, 1, limit=400)[0] - k
    W = float(W_mp(k))
    assert abs(-2 * fp - 0.5 * np.pi * _A(k, W)) < 1e-9


def test_kernels_decay_and_long_time_integrals():
    # Section 3.1: both kernels tend to zero at large argument.  Their time
    # integrals over (0, inf) are -1/2 (shear: matches the radiation-damping
    # coefficient mu/(2 c_s) once multiplied by -mu|k|/(c_s|k|)) and 0
    # (normal).  The integrals converge slowly (oscillating ~T^-1/2), so the
    # running integral is Cesaro-averaged over [X/2, X].
    T = np.linspace(0.0, 1200.0, 1_200_001)
    ct, cn = kernels_fp(T, CS, CP)
    for c, target in ((ct, -0.5), (cn, 0.0)):
        run = np.concatenate([[0.0], np.cumsum(0.5 * (c[1:] + c[:-1]) * np.diff(T))])
        lo = np.searchsorted(T, 600.0)
        assert abs(run[lo:].mean() - target) < 2e-4
    big = T > 150
    assert np.abs(ct[big]).max() < 0.05 and np.abs(cn[big]).max() < 0.15


def test_fp64_evaluator_agrees_with_30_digit_evaluator():
    # The FP64 closed form loses accuracy to cancellation; bound it.
    Ts = np.concatenate([np.linspace(0.01, 5, 7), np.linspace(10, 250, 13)])
    ct_fp, cn_fp = kernels_fp(Ts, CS, CP)
    for i, T in enumerate(Ts):
        ct, cn = kernels_mp(T, CS, CP)
        assert abs(ct_fp[i] - float(ct)) < 3e-9
        assert abs(cn_fp[i] - float(cn)) < 3e-9


def test_fp64_evaluator_is_finite_where_scipy_struve_fails():
    # scipy's Struve functions return NaN near x = 25.7646 (eta T with
    # T = 14.8752 at these wave speeds); the evaluator must not.
    T = np.linspace(14.87, 14.88, 20001)
    ct, cn = kernels_fp(T, CS, CP)
    assert np.all(np.isfinite(ct)) and np.all(np.isfinite(cn))
    ref = kernels_mp(14.87520345, CS, CP)
    v = kernels_fp(np.array([14.87520345]), CS, CP)
    assert abs(v[0][0] - float(ref[0])) < 3e-9 and abs(v[1][0] - float(ref[1])) < 3e-9


def test_golden_kernel_table_is_oracle_output():
    # The stored 30-digit table equals fresh oracle evaluations at spot points.
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "kernel_table_L10km_beta05_N256.npz")
    z = np.load(path)
    for p in (0, 1, 17, 1023, 20000, int(z["p_max"])):
        with mp.workdps(MP_DPS):
            ct, cn = kernels_mp(mp.mpf(repr(float(z["delta"]))) * p, CS, CP)
        assert z["CT"][p] == float(ct) and z["CN"][p] == float(cn)


def test_fp64_w_and_kernels_match_the_30_digit_evaluator():
    """The FP64 evaluator (Neumann series, quadrature of J1(t)/t, and the
    large-argument form J0 A + J1 B) against the 30-digit closed forms of W
    (section 2.3, via Struve functions) and of C^T, C^N, across every branch
    and the branch points."""
    import mpmath as mp
    from oracle.kernels import W_mp, _W_fp, kernels_fp, kernels_mp
    x = np.concatenate([np.linspace(0.0, 60.0, 241), [4.999999, 5.0, 34.999999, 35.0],
                        np.linspace(60.0, 450.0, 40)])
    w = _W_fp(x)
    err = max(abs(w[i] - float(W_mp(v))) for i, v in enumerate(x))
    assert err < 1e-15, err
    T = np.array([0.01, 0.7, 2.0, 6.0, 13.0, 15.7, 20.2, 28.9, 40.0, 100.0, 199.0, 240.0])
    ct, cn = kernels_fp(T, CS, CP)
    for i, t in enumerate(T):
        with mp.workdps(30):
            a, b = kernels_mp(t, CS, CP)
        tol = 1e-15 * max(1.0, t * t)       # the T^2 W terms amplify the rounding of W
        assert abs(ct[i] - float(a)) < tol and abs(cn[i] - float(b)) < tol, t


def _normal_step_response_space_time(T, cs, cp, mu=1.0):
    """sigma_22(0, t) for kappa*du = H(t) sin(k y), by quadrature of the
    flat-fault space-time normal-traction kernel of section 2.4 in the form
    of appendix B (kernels acting on the rate kappa*du_dot, so a step in
    kappa*du gives the bracket itself at lag t):

      P part, |xi| < c_p t:  4 c_s^2 mu t sqrt(t^2 - xi^2/c_p^2) / (2 pi xi^3)
                             + c_s^2 lam^2 t / (2 pi mu c_p^2 xi sqrt(t^2 - xi^2/c_p^2))
      S part, |xi| < c_s t:  -[4 c_s^2 mu t sqrt(t^2 - xi^2/c_s^2) / (2 pi xi^3)
                               + (lam + 2 mu) t / (2 pi xi sqrt(t^2 - xi^2/c_s^2))]

    (Readings: the P coefficient c_s^2 lam^2 / mu of appendix B, whose
    main-text copy lost the 1/mu; the sign of the last term from appendix B's
    bracketed S part.)  sigma(0, t) = -int B(xi, t) sin(k xi) dxi (B is odd,
    the integrand even).  The two xi^-3 terms are combined near xi = 0, where
    their difference is O(1/xi); tanh-sinh quadrature takes the inverse
    square roots at the wave fronts.  Units: k = 1, so c_s t = T."""
    mp.mp.dps = 30
    cs, cp, mu = mp.mpf(cs), mp.mpf(cp), mp.mpf(mu)
    lam = mu * (cp ** 2 / cs ** 2 - 2)
    s = mp.mpf(T) / cs
    A = lambda x: s * s - x * x / cp ** 2
    B = lambda x: s * s - x * x / cs ** 2
    p3 = lambda x: 4 * cs ** 2 * mu * s * mp.sqrt(A(x)) / (2 * mp.pi * x ** 3)
    s3 = lambda x: -4 * cs ** 2 * mu * s * mp.sqrt(B(x)) / (2 * mp.pi * x ** 3)
    p1 = lambda x: cs ** 2 * lam ** 2 * s / (2 * mp.pi * mu * cp ** 2 * x * mp.sqrt(A(x)))
    s1 = lambda x: -(lam + 2 * mu) * s / (2 * mp.pi * x * mp.sqrt(B(x)))
    # p3 + s3 without cancellation: sqrt(A) - sqrt(B) = x^2 (1/cs^2 - 1/cp^2) / (sqrt A + sqrt B)
    ps3 = lambda x: (4 * cs ** 2 * mu * s * (1 / cs ** 2 - 1 / cp ** 2)
                     / (2 * mp.pi * x * (mp.sqrt(A(x)) + mp.sqrt(B(x)))))
    a = cs * s / 2
    I = mp.quad(lambda x: (ps3(x) + p1(x) + s1(x)) * mp.sin(x), [0, a])
    I += mp.quad(lambda x: (p3(x) + s3(x) + p1(x) + s1(x)) * mp.sin(x), [a, cs * s])
    I += mp.quad(lambda x: (p3(x) + p1(x)) * mp.sin(x), [cs * s, cp * s])
    return -2 * I


@pytest.mark.parametrize("cs,cp", [(CS, CP), (3000.0, 6000.0)])
def test_normal_kernel_is_the_transform_of_the_space_time_kernel(cs, cp):
    """Sections 2.4 / appendix B: the normal-traction response to a step of
    kappa*du = sin(k y) from the printed space-time kernel is
    sigma_22 = mu [(1 - r) + C^N_II(c_s k t)] cos(k x) (tension positive),
    so sigma_22(0, t) = mu [(1 - r) + C^N_II].  The oracle's
    compression-positive reading, multiplier -i sgn(k), gives the negative
    of this.  A pin of the dynamic normal operator that does not go through
    the spectral multipliers."""
    r = (cs / cp) ** 2
    for T in ("0.05", "0.5", "2", "7", "20", "60"):
        st = mp.re(_normal_step_response_space_time(mp.mpf(T), cs, cp))
        with mp.workdps(30):
            cn = mp.re(kernels_mp(mp.mpf(T), cs, cp)[1])
            want = (1 - (mp.mpf(cs) / mp.mpf(cp)) ** 2) + cn
        assert abs(st - want) < mp.mpf("1e-15"), (T, st, want)
        fp = kernels_fp(np.array([float(T)]), cs, cp)[1][0]
        # the FP64 evaluator's own bound (its pin above): 1e-15 max(1, T^2)
        assert abs(float(st) - (1 - r) - fp) < 1e-15 * max(1.0, float(T) ** 2), (T, float(st), fp)
