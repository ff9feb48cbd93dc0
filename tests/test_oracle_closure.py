"""Pins of the closure reference (oracle/closure.py and the closure hooks of
the oracle stepper).  The closure is not in the paper: its accuracy against
the plain method is measured, not pinned; these tests pin the network
arithmetic (finite differences, identities, rounding) and the bookkeeping
(the tail plus the kept sum is the full sum)."""

import math

import numpy as np
import pytest

from oracle import closure as cl
from oracle.stepper import OracleFault
from sbiem_inputs import FrictionSpec, friction_fields, rough_fault

MU, CS, CP = 30e9, 3464.0, 6000.0


def test_parameter_count_and_layout():
    assert cl.N_PARAMS == 33 * 64 + 64 + 64 * 64 + 64 + 64 * 2 + 2 == 6466
    p = np.arange(cl.N_PARAMS, dtype=float)
    W1, b1, W2, b2, W3, b3 = cl.unpack(p)
    assert W1[0, 1] == 1 and b1[0] == 33 * 64 and W3.shape == (64, 2) and b3[-1] == 6465
    assert np.array_equal(cl.pack(cl.unpack(p)), p)


def test_gelu_identities():
    z = np.linspace(-6, 6, 101)
    assert cl.gelu(np.array([0.0]))[0] == 0.0
    assert np.allclose(cl.gelu(z) - cl.gelu(-z), z, rtol=0, atol=1e-15)   # erf is odd
    h = 1e-6
    fd = (cl.gelu(z + h) - cl.gelu(z - h)) / (2 * h)
    assert np.max(np.abs(fd - cl.gelu_grad(z))) < 1e-9
    assert abs(cl.gelu_grad(np.array([0.0]))[0] - 0.5) < 1e-15


def test_bfloat16_rounding():
    one = 1.0
    ulp = 2.0 ** -7                       # bfloat16 spacing in [1, 2)
    assert cl.bf16(one) == one
    assert cl.bf16(one + ulp / 2) == one                  # tie to even (mantissa 0)
    assert cl.bf16(one + 1.5 * ulp) == one + 2 * ulp      # tie to even (mantissa 2)
    assert cl.bf16(one + 0.75 * ulp) == one + ulp
    assert cl.bf16(-3.0) == -3.0
    x = np.random.default_rng(3).standard_normal(1000) * 10.0
    r = cl.bf16(x)
    # 8 significant bits: relative error at most half a unit of 2^-7
    assert np.max(np.abs(r - x) / np.abs(x)) <= 2.0 ** -8 * (1 + 1e-12)


def test_backward_matches_central_differences():
    rng = np.random.default_rng(5)
    p = cl.init_params(1) + 0.05 * rng.standard_normal(cl.N_PARAMS)
    x = rng.standard_normal((7, 33))
    t = rng.standard_normal((7, 2))
    _, g = cl.loss_and_grad(p, x, t)
    idx = np.concatenate([rng.choice(cl.N_PARAMS, 300, replace=False),
                          np.arange(33 * 64, 33 * 64 + 64), np.arange(cl.N_PARAMS - 2, cl.N_PARAMS)])
    h = 1e-6
    for i in idx:
        e = np.zeros(cl.N_PARAMS)
        e[i] = h
        fd = (cl.loss_and_grad(p + e, x, t)[0] - cl.loss_and_grad(p - e, x, t)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(g[i])), (i, fd, g[i])


def test_first_adam_step_moves_every_parameter_by_lr_times_sign():
    rng = np.random.default_rng(6)
    p = cl.init_params(2)
    x = rng.standard_normal((32, 33))
    t = rng.standard_normal((32, 2))
    _, g = cl.loss_and_grad(p, x[:8], t[:8])
    lr = 1e-3
    p1, m, v, step, losses = cl.adam_steps(p, np.zeros_like(p), np.zeros_like(p), 0, x, t, 8, 1, lr)
    big = np.abs(g) > 1e-4
    assert step == 1 and losses.shape == (1,)
    assert np.allclose((p1 - p)[big], -lr * np.sign(g[big]), rtol=1e-3, atol=0)


def test_training_reduces_the_loss_on_a_learnable_target():
    rng = np.random.default_rng(7)
    x = rng.standard_normal((512, 33))
    t = np.stack([np.tanh(x[:, 1] + 0.5 * x[:, 2]), 0.3 * x[:, 0] * x[:, 3]], axis=1)
    p = cl.init_params(3)
    L0 = cl.loss_and_grad(p, x, t)[0]
    p, m, v, step, losses = cl.adam_steps(p, np.zeros_like(p), np.zeros_like(p), 0, x, t, 64, 400, 3e-3)
    assert cl.loss_and_grad(p, x, t)[0] < 0.1 * L0


def _fault(N=256, L=10e3, steps=80, seed=3):
    spec = FrictionSpec(overstress=9e6, w_nuc=800.0)
    fr = friction_fields(N, L, MU, CS, spec)
    dt = 0.5 * L / N / CS
    f = OracleFault(N, L, MU, CS, CP, dt=dt, friction=fr, h=rough_fault(N, L, 3e-3, seed),
                    theta_mode="exp", transform="fft")
    f.run(steps)
    return f


def test_tail_plus_kept_sum_is_the_full_history_sum():
    f = _fault()
    smp = f.closure_samples(0.25)
    assert len(smp["mode"]) > 0
    Mk, use = cl.kept_lags(f.w.M, 0.25)
    ST, SN = f.history_sums()
    for n, kind, tail in zip(smp["mode"], smp["kind"], smp["tail"]):
        H = f.HT if kind == 0 else f.HN
        w = f.w.wT if kind == 0 else f.w.wN
        kept = sum(w[f.w.off[n] + j] * H[f.hoff[n] + j - 1] for j in range(1, Mk[n]))
        full = (ST if kind == 0 else SN)[n]
        assert abs(kept + tail - full) <= 1e-12 * max(abs(full), 1e-300)


def test_closure_inputs_are_scale_free():
    f = _fault(steps=60)
    smp = f.closure_samples(0.25)
    x, r = smp["x"], smp["r"]
    assert np.allclose(np.mean(x[:, 1:] ** 2, axis=1) * 2, 1.0)   # unit RMS of the 16 values
    # doubling every history value doubles r and leaves x unchanged
    f.HT *= 2.0
    f.HN *= 2.0
    smp2 = f.closure_samples(0.25)
    assert np.allclose(smp2["x"], x, rtol=1e-14, atol=1e-15)
    assert np.allclose(smp2["r"], 2 * r, rtol=1e-14)
    assert np.allclose(smp2["y"], smp["y"], rtol=1e-12, atol=1e-15)


def test_kept_lags_rule():
    M = np.array([1, 40, 68, 69, 70, 400, 1000])
    Mk, use = cl.kept_lags(M, 0.25)
    assert list(use) == [False, False, False, True, True, True, True]
    assert list(Mk) == [1, 40, 68, 18, 18, 100, 250]


def test_zero_network_closure_is_exact_for_a_history_constant_beyond_the_cut():
    """With y = 0 the tail is D a_15: exact when every discarded lag holds the
    oldest kept value (the kept lags may hold anything)."""
    N, L = 256, 10e3
    spec = FrictionSpec(overstress=9e6, w_nuc=800.0)
    fr = friction_fields(N, L, MU, CS, spec)
    dt = 0.5 * L / N / CS
    h = rough_fault(N, L, 3e-3, 4)
    zero = np.zeros(cl.N_PARAMS)
    plain = OracleFault(N, L, MU, CS, CP, dt=dt, friction=fr, h=h, transform="fft")
    clo = OracleFault(N, L, MU, CS, CP, dt=dt, friction=fr, h=h, transform="fft", closure=(zero, zero, 0.25))
    assert clo.closed.sum() > 20
    rng = np.random.default_rng(11)
    for kind in (0, 1):
        Hp = plain.HT if kind == 0 else plain.HN
        Hc = clo.HT if kind == 0 else clo.HN
        for n in range(1, N // 2 + 1):
            kept = rng.standard_normal(plain.hM[n]) + 1j * rng.standard_normal(plain.hM[n])
            if n == N // 2:
                kept = kept.real + 0j
            Mk = int(clo.M_kept[n]) if clo.closed[n] else int(plain.w.M[n])
            kept[Mk - 1:] = kept[Mk - 2] if Mk >= 2 else kept[0]     # lags >= M'-1 equal a_15
            for m, vals in ((n, kept), (N - n, np.conj(kept))):
                if m == N // 2 and n != N // 2:
                    continue
                Hp[plain.hoff[m]:plain.hoff[m] + plain.hM[m]] = vals
                Hc[clo.hoff[m]:clo.hoff[m] + clo.hM[m]] = vals[:clo.hM[m]]
    ST_p, SN_p = plain.history_sums()
    ST_c, SN_c = clo.history_sums()
    for a, b in ((ST_c, ST_p), (SN_c, SN_p)):
        assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b))
    # and truncation alone (dropping the tail) is far from it
    tT, tN = clo.closure_tails()
    assert np.max(np.abs(ST_c - tT - ST_p)) > 1e-3 * np.max(np.abs(ST_p))
