"""GPU parity on the paths that long runs and full-size workloads take, and
on the boundary's failure and allocator paths (through the C ABI).

* Windows longer than one convolution task (8192 FP32 or 4096 FP64 ring
  records) are split into pieces whose partial sums the mode stage adds;
  here every piece carries history, and the ring has wrapped.
* The FP32 step is compared after its ring has wrapped, through a rupture.
* A batch of faults of uneven N is compared with the oracle member by member.
* Tolerances as in test_gpu_parity.py, in the plain norm-wise relative
  measure ||gpu - oracle||_inf / ||oracle||_inf: 1e-10 in FP64, 1e-5 on the
  FP32 path's tractions.
"""

import numpy as np
import pytest

from scenarios import CS, CP, MU, NU, Scenario, fields, make_oracle, make_plan, rel, rough_10km
from sbiem_inputs import FrictionSpec

pytestmark = pytest.mark.gpu


def _pkg():
    import paper_2107_03550_amd as pkg
    return pkg


def _random_history(N, nt, seed, scale=1e-3):
    """Slip snapshots whose interval rates are random in space and time."""
    rng = np.random.default_rng(seed)
    x = np.arange(N) / N
    rates = rng.random((nt, N)) * scale * (1 + np.cos(2 * np.pi * x))[None, :]
    base = 0.3 * scale * (1.0 + 0.5 * np.sin(2 * np.pi * 3 * x) + 0.2 * rng.standard_normal(N))
    return np.vstack([np.zeros((1, N)), np.cumsum(rates, axis=0)]) + base[None, :]


def _low_mode_history(N, nt, seed, noise=1e-9):
    """Slip snapshots whose rates live in wavenumbers 1 and 2 (smooth random
    time histories), plus white noise of relative size ``noise``.  The kernel
    arguments of those modes stay below 4 pi over their whole window, where
    the oracle's FP64 closed-form kernels are exact to about 1e-13, so the
    comparison can be held at the FP64 tolerance with long windows."""
    rng = np.random.default_rng(seed)
    x = np.arange(N) / N
    t = np.arange(nt) / nt
    rates = np.zeros((nt, N))
    for m in (1, 2):
        amp = 0.5 + sum(rng.uniform(0.1, 0.4) * np.sin(2 * np.pi * rng.uniform(1, 9) * t
                                                        + rng.uniform(0, 6.3)) for _ in range(3))
        rates += amp[:, None] * np.cos(2 * np.pi * m * x + rng.uniform(0, 6.3))[None, :]
    rates = 1e-3 * (rates + noise * rng.standard_normal((nt, N)))
    base = 2e-4 * np.cos(2 * np.pi * x + 0.4)
    return np.vstack([np.zeros((1, N)), np.cumsum(rates, axis=0)]) + base[None, :]


def _pieces(M, task_records):
    """Convolution pieces of a window of M lags (ring of M - 1 records)."""
    return -(-(M - 1) // task_records)


@pytest.mark.parametrize("tile", [0, 64, 320])
def test_stress_fp32_long_windows_in_three_pieces(tile):
    """N = 64 at beta = 1/320: every window holds about 20480 lags, three
    FP32 tasks of 8192 ring records (tile 64: packed rows, a mode across
    three or four 128-row tasks; tile 320: tasks of 10240 records, two or
    three pieces); 21000 intervals fill every record (the fill wraps) with
    random rates."""
    from oracle.spectral import curvature_fft
    from oracle.stress import stress_from_history
    from oracle.windows import midpoint_weights
    pkg = _pkg()
    N, beta = 64, 1.0 / 320.0
    L = 10.0 * N
    dt = beta * (L / N) / CS
    nt = 21000
    h = rough_10km(N, seed=11, alpha=5e-3) * (L / 10e3)
    p = pkg.Plan(N, L, MU, NU, CS, CP, h)
    p.set_precision(pkg.SBIEM_FP32CONV)
    p.set_conv_tile(tile)
    M = p.window_lengths(dt)
    assert M.min() > 16385 and _pieces(M.max(), 8192) == 3 and nt > M.max()
    hist = _random_history(N, nt, seed=21)
    tau, sig = p.stress(hist, dt)
    w = midpoint_weights(N, L, CS, CP, dt)
    rt, rs = stress_from_history(hist, dt, L, MU, CS, CP, curvature_fft(h, L), w, transform="fft")
    print("fp32 three-piece windows (tile %d):" % tile, rel(tau, rt), rel(sig, rs))
    assert rel(tau, rt) < 1e-5 and rel(sig, rs) < 1e-5, (rel(tau, rt), rel(sig, rs))


def test_stress_fp64_long_windows_in_three_pieces():
    """N = 64 at beta = 1/160: windows of about 10240 lags, three FP64 tasks
    of 4096 ring records; 11000 intervals (the fill wraps).  The oracle takes
    the library's curvature as data, so only the hot path is compared."""
    from oracle.stress import stress_from_history
    from oracle.windows import midpoint_weights
    pkg = _pkg()
    N, beta = 64, 1.0 / 160.0
    L = 10.0 * N
    dt = beta * (L / N) / CS
    nt = 11000
    h = rough_10km(N, seed=12, alpha=5e-3) * (L / 10e3)
    p = pkg.Plan(N, L, MU, NU, CS, CP, h)
    M = p.window_lengths(dt)
    assert M[0] == 160 * N and _pieces(M[0], 4096) == 3 and nt > M[0]
    hist = _low_mode_history(N, nt, seed=22)
    tau, sig = p.stress(hist, dt)
    w = midpoint_weights(N, L, CS, CP, dt)
    rt, rs = stress_from_history(hist, dt, L, MU, CS, CP, p.get_curvature(), w, transform="fft")
    print("fp64 three-piece windows:", rel(tau, rt), rel(sig, rs))
    assert rel(tau, rt) < 1e-10 and rel(sig, rs) < 1e-10, (rel(tau, rt), rel(sig, rs))


def test_step_fp32_past_the_window_through_a_rupture():
    """FP32 steps of an N = 512 fault (M_max = 1024) for 1100 steps through
    a rupture: the ring wraps and the FP32 lag/phase arithmetic of the
    convolution is exercised on every slot."""
    pkg = _pkg()
    N = 512
    L = 10.0 * N
    sc = Scenario(N, L, 0.5 * (L / N) / CS, rough_10km(N, seed=13, alpha=3e-3) * (L / 10e3),
                  spec=FrictionSpec(overstress=9e6, w_nuc=600.0), theta_mode="exp",
                  consistent_V0=True)
    p = make_plan(sc, pkg.SBIEM_FP32CONV)
    assert p.window_lengths(sc.dt).max() == 2 * N
    from oracle.stepper import OracleFault
    o = OracleFault(sc.N, sc.L, MU, CS, CP, dt=sc.dt, friction=fields(sc), h=sc.h,
                    theta_mode=sc.theta_mode, transform="fft")
    worst = {k: 0.0 for k in ("tau_el", "sigma_el", "slip", "V")}
    vmax = 0.0
    for _ in range(11):
        p.run(sc.dt, 100)
        o.run(100)
        g = p.get_state()
        vmax = max(vmax, o.V.max())
        for k, ref in (("slip", o.slip), ("V", o.V), ("tau_el", o.tau_el),
                       ("sigma_el", o.sigma_el)):
            worst[k] = max(worst[k], rel(g[k], ref))
    print("fp32 1100 steps through a rupture:", worst, "max V", vmax)
    assert p.steps_done() == 1100 and vmax > 0.1
    assert worst["tau_el"] < 1e-5 and worst["sigma_el"] < 1e-5, worst


def test_batch_of_uneven_faults_matches_oracle():
    """A batch of three faults (N = 256, 512, 1024; the first one's ring wraps
    twice) against the oracle of each member."""
    from oracle.stepper import OracleFault
    pkg = _pkg()
    dt = 0.5 * 10.0 / CS
    scs = []
    for N, seed in ((256, 31), (512, 32), (1024, 33)):
        L = 10.0 * N
        scs.append(Scenario(N, L, dt, rough_10km(N, seed=seed, alpha=4e-3) * (L / 10e3),
                            spec=FrictionSpec(overstress=8e6, w_nuc=300.0), theta_mode="exp",
                            consistent_V0=True))
    plans = [make_plan(sc, pkg.SBIEM_FP32CONV) for sc in scs]
    orcs = [OracleFault(sc.N, sc.L, MU, CS, CP, dt=sc.dt, friction=fields(sc), h=sc.h,
                        theta_mode=sc.theta_mode, transform="fft") for sc in scs]
    batch = pkg.Batch(plans)
    worst = [0.0] * len(scs)
    for _ in range(4):
        batch.run(150)
        for i, (p, o) in enumerate(zip(plans, orcs)):
            o.run(150)
            g = p.get_state()
            worst[i] = max(worst[i], rel(g["tau_el"], o.tau_el), rel(g["sigma_el"], o.sigma_el))
    print("uneven batch vs oracle (tractions):", worst)
    batch.close()
    assert max(worst) < 1e-5, worst


def test_stress_fp32_full_size_plain_norm():
    """sbiem_stress at N = 65536 (the rough-N65536 fault) over 24 intervals
    of random-sign rates from zero slip: at all but the lowest wavenumbers
    the dynamic part of each interval has decayed well before the end, so
    the tractions are not a cancellation of static and dynamic parts; the
    comparison is in the plain norm."""
    from oracle.spectral import curvature_fft
    from oracle.stress import stress_from_history
    from oracle.windows import midpoint_weights
    from sbiem_inputs import workload
    pkg = _pkg()
    w = workload("rough-N65536")
    nt = 24
    rng = np.random.default_rng(41)
    rates = 1e-3 * rng.standard_normal((nt, w.N))
    hist = np.vstack([np.zeros((1, w.N)), np.cumsum(rates, axis=0) * w.dt])
    p = pkg.Plan(w.N, w.L, w.mu, w.nu, w.cs, w.cp, w.h)
    p.set_precision(pkg.SBIEM_FP32CONV)
    tau, sig = p.stress(hist, w.dt)
    wts = midpoint_weights(w.N, w.L, w.cs, w.cp, w.dt, max_lag=nt)
    rt, rs, st, ss = stress_from_history(hist, w.dt, w.L, w.mu, w.cs, w.cp,
                                         curvature_fft(w.h, w.L), wts, transform="fft", parts=True)
    print("N=65536 stress, plain norm:", rel(tau, rt), rel(sig, rs),
          "| max |tau|, |static|, |dynamic|:", np.abs(rt).max(), np.abs(st).max(),
          np.abs(rt - st).max())
    assert rel(tau, rt) < 1e-5 and rel(sig, rs) < 1e-5, (rel(tau, rt), rel(sig, rs))


def test_torch_caching_allocator_backs_a_plan():
    """Plan memory routed through torch's caching allocator: the allocator
    is called, and the steps equal those of a plan on hipMalloc bit for bit."""
    import torch
    pkg = _pkg()
    sc = Scenario(512, 10e3, 0.5 * (10e3 / 512) / CS, rough_10km(512, seed=5), theta_mode="exp",
                  spec=FrictionSpec(overstress=8e6), consistent_V0=True)
    ref = make_plan(sc, pkg.SBIEM_FP32CONV)
    ref.run(sc.dt, 40)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    pkg.set_torch_allocator()
    try:
        p = make_plan(sc, pkg.SBIEM_FP32CONV)
        held = torch.cuda.memory_allocated() - before
        p.run(sc.dt, 40)
        g, r = p.get_state(), ref.get_state()
        p.close()
        after = torch.cuda.memory_allocated() - before
    finally:
        pkg.set_default_allocator()
    print("bytes held through torch's allocator:", held, "after destroy:", after)
    assert held > 0 and after == 0
    for k in ("slip", "V", "theta", "tau_el", "sigma_el"):
        assert np.array_equal(g[k], r[k]), k


def test_failures_forced_from_the_host():
    """SBIEM_ENOTREADY before friction and state; SBIEM_ENEWTON with a
    one-iteration Newton limit; SBIEM_ESTATE from the paper's explicit state
    update at V dt / Dc > 2.  Each failing step leaves the state at the start
    of the step, and the run continues once the cause is removed."""
    pkg = _pkg()
    N, L = 64, 10e3
    dt = 0.5 * (L / N) / CS
    bare = pkg.Plan(N, L, MU, NU, CS, CP)
    assert bare.run_status(dt, 1) == -7
    sc = Scenario(N, L, dt, rough_10km(N, seed=5, alpha=3e-3), theta_mode="exp",
                  spec=FrictionSpec(overstress=3e6), consistent_V0=True)
    p = make_plan(sc, pkg.SBIEM_FP64)
    q = make_plan(sc, pkg.SBIEM_FP64)
    p.run(dt, 5)
    q.run(dt, 10)
    before = p.get_state()
    p.set_newton_limit(1)
    assert p.run_status(dt, 3) == -4
    cnt, idx = p.failures()
    assert cnt > 0 and 0 <= idx < N and p.steps_done() == 5
    after = p.get_state()
    for k in ("slip", "V", "theta"):
        assert np.array_equal(before[k], after[k]), k
    p.set_newton_limit(0)
    p.run(dt, 5)
    g, r = p.get_state(), q.get_state()
    for k in ("slip", "V", "theta", "tau_el", "sigma_el"):
        assert rel(g[k], r[k]) < 1e-12, (k, rel(g[k], r[k]))
    # explicit state update with V dt / Dc = 5.6: theta_p = theta (1 - 5.6) + dt < 0
    fr = fields(sc)
    s = make_plan(Scenario(N, L, dt, sc.h, theta_mode="paper", spec=sc.spec), pkg.SBIEM_FP64)
    s.set_state(fr["slip0"], np.full(N, 1.0), np.full(N, 1.0), 0.0)
    assert s.run_status(dt, 1) == -5
    assert s.failures()[0] == N and s.steps_done() == 0
