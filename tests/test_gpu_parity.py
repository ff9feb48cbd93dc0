"""GPU parity of the HIP path against the CPU oracle (through the C ABI).

Tolerances (norm-wise relative, max over the compared steps): 1e-10 in
FP64; 1e-5 on tau^el and sigma^el in the FP32 convolution path.
"""

import numpy as np
import pytest

from scenarios import (DT_10KM, Scenario, golden_table, make_oracle, make_plan, rel,
                       rel_parts, rough_10km, seamount_h, MU, NU, CS, CP)
from sbiem_inputs import FrictionSpec

pytestmark = pytest.mark.gpu


def _pkg():
    import paper_2107_03550_amd as pkg
    return pkg


def _history(N, nt, seed, scale=1e-3):
    rng = np.random.default_rng(seed)
    x = np.arange(N) / N
    rates = rng.random((nt, N)) * scale * (1 + np.cos(2 * np.pi * x))[None, :]
    base = 0.3 * scale * (1.0 + 0.5 * np.sin(2 * np.pi * 3 * x) + 0.2 * rng.standard_normal(N))
    return np.vstack([np.zeros((1, N)), np.cumsum(rates, axis=0)]) + base[None, :]


# ---------------------------------------------------------------- windows
@pytest.mark.parametrize("N,L", [(256, 10e3), (8192, 80e3), (1024, 10240.0)])
def test_window_lengths_match_oracle(N, L):
    from oracle.windows import window_steps
    pkg = _pkg()
    p = pkg.Plan(N, L, MU, NU, CS, CP)
    dt = 0.5 * L / N / CS
    M = p.window_lengths(dt)
    ref = window_steps(N, L, CS, dt)[1:N // 2 + 1]
    assert np.array_equal(M, ref)


# ---------------------------------------------------------------- stress path
@pytest.mark.parametrize("N,nt", [(32, 600), (256, 700), (256, 3), (64, 0), (64, 1)])
def test_stress_fp64_matches_oracle(N, nt):
    from oracle.spectral import curvature
    from oracle.stress import stress_from_history
    from oracle.windows import midpoint_weights
    pkg = _pkg()
    L, dt = 10e3, DT_10KM
    h = rough_10km(N, seed=4, alpha=3e-3)
    hist = _history(N, nt, seed=N + nt)
    p = pkg.Plan(N, L, MU, NU, CS, CP, h)
    tau, sig = p.stress(hist, dt)
    w = midpoint_weights(N, L, CS, CP, dt, golden_table())
    rt, rs = stress_from_history(hist, dt, L, MU, CS, CP, curvature(h, L), w)
    assert rel(tau, rt) < 1e-10 and rel(sig, rs) < 1e-10, (rel(tau, rt), rel(sig, rs))


@pytest.mark.parametrize("N,nt,tile", [(1024, 300, 0), (512, 1100, 0), (1024, 1500, 256),
                                        (1024, 1500, 320), (256, 2100, 320),
                                        (1024, 1500, 1024), (1024, 1500, 64), (512, 300, 64),
                                        (256, 2100, 64)])
def test_stress_fp32_matches_oracle(N, nt, tile):
    """FP32 stress path against the oracle; the later cases put windows of up
    to 2048 records through tiles of 256, 320 and 1024 records and through packed
    rows (tile 64: modes of one to 32 rows sharing waves and tasks, a mode
    cut by a task boundary, a padded last task)."""
    from oracle.spectral import curvature
    from oracle.stress import stress_from_history
    from oracle.windows import midpoint_weights
    pkg = _pkg()
    L = 10.0 * N
    dt = 0.5 * (L / N) / CS
    h = rough_10km(N, seed=9, alpha=5e-3) * (L / 10e3)
    hist = _history(N, nt, seed=nt)
    p = pkg.Plan(N, L, MU, NU, CS, CP, h)
    p.set_precision(pkg.SBIEM_FP32CONV)
    p.set_conv_tile(tile)
    tau, sig = p.stress(hist, dt)
    w = midpoint_weights(N, L, CS, CP, dt)
    rt, rs = stress_from_history(hist, dt, L, MU, CS, CP, curvature(h, L), w)
    assert rel(tau, rt) < 1e-5 and rel(sig, rs) < 1e-5, (rel(tau, rt), rel(sig, rs))


# ---------------------------------------------------------------- time step
def test_step_fp64_rough_N256_2000_steps():
    """The N = 256 rough-fault FP64 workload, 2000 fixed steps."""
    pkg = _pkg()
    sc = Scenario(256, 10e3, DT_10KM, rough_10km(256, seed=0, alpha=1e-3))
    p = make_plan(sc, pkg.SBIEM_FP64)
    o = make_oracle(sc, golden_table())
    worst = {k: 0.0 for k in ("slip", "V", "theta", "tau_el", "sigma_el")}
    done = 0
    for chunk in (1, 9, 90, 400, 500, 1000):
        p.run(sc.dt, chunk)
        o.run(chunk)
        done += chunk
        g = p.get_state()
        ref = dict(slip=o.slip, V=o.V, theta=o.theta, tau_el=o.tau_el, sigma_el=o.sigma_el)
        for k in worst:
            worst[k] = max(worst[k], rel(g[k], ref[k]))
        assert abs(g["t"] - o.t) < 1e-9
    assert done == 2000 and p.steps_done() == 2000
    assert all(v < 1e-10 for v in worst.values()), worst


def test_step_fp64_dynamic_rupture():
    """Strong overstress: slip rates up to m/s, exact theta update."""
    pkg = _pkg()
    spec = FrictionSpec(overstress=9e6, w_nuc=1500.0)
    sc = Scenario(128, 10e3, DT_10KM, rough_10km(128, seed=2, alpha=3e-3), spec=spec,
                  theta_mode="exp", consistent_V0=True)
    p = make_plan(sc, pkg.SBIEM_FP64)
    # the library's curvature as data: the comparison measures the step alone
    o = make_oracle(sc, golden_table(), kappa=p.get_curvature())
    worst = 0.0
    for _ in range(6):
        p.run(sc.dt, 50)
        o.run(50)
        g = p.get_state()
        for k, ref in (("slip", o.slip), ("V", o.V), ("tau_el", o.tau_el), ("sigma_el", o.sigma_el)):
            worst = max(worst, rel(g[k], ref))
    print("fp64 rupture worst relative error", worst, "max V", o.V.max())
    assert o.V.max() > 1e-2
    assert worst < 1e-10, worst


@pytest.mark.parametrize("tile", [0, 64, 320])
def test_step_fp32_dynamic_rupture_N1024(tile):
    pkg = _pkg()
    N = 1024
    L = 10.0 * N
    spec = FrictionSpec(overstress=9e6, w_nuc=1500.0)
    h = rough_10km(N, seed=3, alpha=3e-3) * (L / 10e3)
    sc = Scenario(N, L, 0.5 * (L / N) / CS, h, spec=spec, theta_mode="exp", consistent_V0=True)
    p = make_plan(sc, pkg.SBIEM_FP32CONV)
    p.set_conv_tile(tile)
    o = make_oracle(sc)
    worst = {"tau_el": 0.0, "sigma_el": 0.0, "slip": 0.0, "V": 0.0}
    # rupture arrival: the first 2-step chunk after which V >= 1e-3 m/s;
    # the other fields compared every 50 steps
    arr_g = np.full(N, -1)
    arr_o = np.full(N, -1)
    for c in range(100):
        p.run(sc.dt, 2)
        o.run(2)
        g = p.get_state()
        arr_g[(arr_g < 0) & (g["V"] >= 1e-3)] = c
        arr_o[(arr_o < 0) & (o.V >= 1e-3)] = c
        if (c + 1) % 25 == 0:
            for k, ref in (("slip", o.slip), ("V", o.V), ("tau_el", o.tau_el),
                           ("sigma_el", o.sigma_el)):
                worst[k] = max(worst[k], rel(g[k], ref))
    reached = arr_o >= 0
    print("fp32 N=1024 rupture (tile %d) worst relative errors" % tile, worst,
          "arrivals: %d elements, %d differ by one 2-step chunk" %
          (reached.sum(), np.count_nonzero(arr_g[reached] != arr_o[reached])))
    assert worst["tau_el"] < 1e-5 and worst["sigma_el"] < 1e-5, worst
    # the rupture spreads over a tenth of the fault or more, and every element
    # ruptures in the same 2-step chunk as in the FP64 oracle (or a
    # neighbouring one, where its V crosses the threshold within rounding of a
    # chunk's end)
    assert reached.sum() > N // 10
    assert np.array_equal(arr_g >= 0, reached)
    assert np.abs(arr_g[reached] - arr_o[reached]).max() <= 1


# ---------------------------------------------------------------- engine properties
def test_run_with_graph_equals_single_steps_bitwise():
    pkg = _pkg()
    sc = Scenario(256, 10e3, DT_10KM, rough_10km(256, seed=1), theta_mode="exp",
                  spec=FrictionSpec(overstress=8e6), consistent_V0=True)
    a = make_plan(sc, pkg.SBIEM_FP32CONV)
    b = make_plan(sc, pkg.SBIEM_FP32CONV)
    a.run(sc.dt, 37)            # two graph replays + 5 single launches
    for _ in range(37):
        b.step(sc.dt)
    ga, gb = a.get_state(), b.get_state()
    for k in ("slip", "V", "theta", "tau_el", "sigma_el"):
        assert np.array_equal(ga[k], gb[k]), k


def _timed_steps(nsteps, graph_steps=16, graphs=2):
    """Steps a profiled run launches directly (with events): one, then up to
    `graphs` graphs of graph_steps steps while that many remain, repeated."""
    timed = 0
    while nsteps > 0:
        timed += 1
        nsteps -= 1
        for _ in range(graphs):
            if nsteps >= graph_steps:
                nsteps -= graph_steps
    return timed


def test_profiled_run_equals_plain_run_bitwise():
    """Profiled runs (one step in 33 launched directly with timing events
    around its conv launch, the others from the step graph) compute exactly
    what graph replays do, and time the direct steps' launches."""
    pkg = _pkg()
    sc = Scenario(256, 10e3, DT_10KM, rough_10km(256, seed=4), theta_mode="exp",
                  spec=FrictionSpec(overstress=8e6), consistent_V0=True)
    a = make_plan(sc, pkg.SBIEM_FP32CONV)
    b = make_plan(sc, pkg.SBIEM_FP32CONV)
    a.set_profiling(True)
    a.run(sc.dt, 67)
    ms, n, nbytes = a.profile()
    assert _timed_steps(67) == 3
    assert n == 3 and ms > 0.0 and nbytes > 0.0
    b.run(sc.dt, 67)
    ga, gb = a.get_state(), b.get_state()
    for k in ("slip", "V", "theta", "tau_el", "sigma_el"):
        assert np.array_equal(ga[k], gb[k]), k


def test_failure_leaves_state_at_start_of_step():
    pkg = _pkg()
    sc = Scenario(64, 10e3, DT_10KM, rough_10km(64, seed=5, alpha=5e-2))
    p = make_plan(sc, pkg.SBIEM_FP64)
    p.run(sc.dt, 3)
    before = p.get_state()
    fr_sigma = np.full(64, 1.0)     # nearly no normal load: the curvature term opens the fault
    from scenarios import fields
    fr = fields(sc)
    # a large slip makes the normal traction change exceed the tiny load
    p.set_friction(fr["a"], fr["b"], fr["Dc"], fr["V_ref"], fr["f0"], -fr_sigma,
                   fr["tau_load"], 0.0, fr["V_pl"])
    st = p.run_status(sc.dt, 20)
    assert st == -6
    cnt, idx = p.failures()
    assert cnt > 0 and 0 <= idx < 64
    after = p.get_state()
    assert p.steps_done() == 3
    for k in ("slip", "V", "theta"):
        assert np.array_equal(before[k], after[k])


@pytest.mark.parametrize("tile", [0, 64, 320])
def test_batch_matches_individual_plans_bitwise(tile):
    pkg = _pkg()
    plans_a, plans_b = [], []
    for N, seed in ((256, 1), (1024, 2), (512, 3)):
        L = 10.0 * N
        sc = Scenario(N, L, 0.5 * 10.0 / CS, rough_10km(N, seed=seed, alpha=4e-3) * (L / 10e3),
                      spec=FrictionSpec(overstress=8e6, w_nuc=300.0), theta_mode="exp",
                      consistent_V0=True)
        plans_a.append(make_plan(sc, pkg.SBIEM_FP32CONV))
        plans_b.append(make_plan(sc, pkg.SBIEM_FP32CONV))
        if tile:
            plans_a[-1].set_conv_tile(tile)
            plans_b[-1].set_conv_tile(tile)
    dt = 0.5 * 10.0 / CS
    batch = pkg.Batch(plans_a)
    batch.run(40)
    for p in plans_b:
        p.run(dt, 40)
    for pa, pb in zip(plans_a, plans_b):
        ga, gb = pa.get_state(), pb.get_state()
        for k in ("slip", "V", "theta", "tau_el", "sigma_el"):
            assert np.array_equal(ga[k], gb[k]), k
    batch.close()


# ---------------------------------------------------------------- full sizes
def _workload_plan_and_oracle(w, nsteps):
    """A plan of workload ``w`` as bench.py builds it, and the oracle on the
    same inputs (numpy FFT as the transform, weights for nsteps lags)."""
    from oracle.stepper import OracleFault
    from sbiem_inputs import friction_fields
    pkg = _pkg()
    fr = friction_fields(w.N, w.L, w.mu, w.cs, w.friction)
    p = pkg.Plan(w.N, w.L, w.mu, w.nu, w.cs, w.cp, w.h)
    p.set_precision(pkg.SBIEM_FP32CONV)
    p.set_friction(fr["a"], fr["b"], fr["Dc"], fr["V_ref"], fr["f0"], fr["sigma_load"],
                   fr["tau_load"], fr["tau_load_rate"], fr["V_pl"])
    p.set_state(fr["slip0"], fr["V0"], fr["theta0"], 0.0)
    p.set_dt(w.dt)
    o = OracleFault(w.N, w.L, w.mu, w.cs, w.cp, dt=w.dt, friction=fr, h=w.h,
                    transform="fft", max_lag=nsteps)
    return p, o


@pytest.mark.parametrize("name,tile", [("seamount-N8192", 0), ("ensemble64-N16384", 0),
                                       ("rough-N65536", 0), ("ensemble16-N262144", 0),
                                       ("rough-N65536", 64), ("ensemble16-N262144", 64),
                                       ("ensemble16-N262144", 320)])
def test_step_fp32_full_size_matches_oracle(name, tile):
    """The first 20 steps of the full-size workloads (graph replay, as in
    bench.py) against the oracle, compared after a 16-step graph replay and
    after 4 single steps.  The tractions are then tiny (the fault is still
    near steady state), the sum of much larger static and dynamic parts, so
    the FP32 gate of 1e-5 is taken relative to the larger part."""
    from sbiem_inputs import ensemble_members, workload
    if name == "ensemble16-N262144":
        w = ensemble_members(name)[0]
    elif name == "ensemble64-N16384":
        w = [m for m in ensemble_members("ensemble64") if m.N == 16384][0]
    else:
        w = workload(name)
    p, o = _workload_plan_and_oracle(w, 20)
    p.set_conv_tile(tile)
    worst = {"tau_el": 0.0, "sigma_el": 0.0, "slip": 0.0, "V": 0.0,
             "tau_el_plain": 0.0, "sigma_el_plain": 0.0}
    for chunk in (16, 4):
        p.run(w.dt, chunk)
        o.run(chunk)
        g = p.get_state()
        for k, ref in (("slip", o.slip), ("V", o.V)):
            worst[k] = max(worst[k], rel(g[k], ref))
        worst["tau_el"] = max(worst["tau_el"], rel_parts(g["tau_el"], o.tau_el, o.tau_static))
        worst["sigma_el"] = max(worst["sigma_el"], rel_parts(g["sigma_el"], o.sigma_el, o.sigma_static))
        worst["tau_el_plain"] = max(worst["tau_el_plain"], rel(g["tau_el"], o.tau_el))
        worst["sigma_el_plain"] = max(worst["sigma_el_plain"], rel(g["sigma_el"], o.sigma_el))
    print(name, "tile", tile, "worst relative errors", worst)
    assert worst["tau_el"] < 1e-5 and worst["sigma_el"] < 1e-5, worst
    assert worst["slip"] < 1e-10 and worst["V"] < 1e-10, worst


def test_stress_fp32_full_size_N262144():
    """sbiem_stress at N = 262144 (two elements per thread in the element
    stage, four slots per thread in the mode stage) against the oracle."""
    from oracle.spectral import curvature_fft
    from oracle.stress import stress_from_history
    from oracle.windows import midpoint_weights
    from sbiem_inputs import ensemble_members
    pkg = _pkg()
    w = ensemble_members("ensemble16-N262144")[1]
    nt = 5
    hist = _history(w.N, nt, seed=9)
    p = pkg.Plan(w.N, w.L, w.mu, w.nu, w.cs, w.cp, w.h)
    p.set_precision(pkg.SBIEM_FP32CONV)
    tau, sig = p.stress(hist, w.dt)
    wts = midpoint_weights(w.N, w.L, w.cs, w.cp, w.dt, max_lag=nt)
    kappa = curvature_fft(w.h, w.L)
    # the library's curvature (extended precision) and numpy's FFT agree to
    # the double-precision amplification of rounding by k^2
    assert rel(p.get_curvature(), kappa) < 1e-9
    rt, rs, st, ss = stress_from_history(hist, w.dt, w.L, w.mu, w.cs, w.cp, kappa, wts,
                                         transform="fft", parts=True)
    et, es = rel_parts(tau, rt, st), rel_parts(sig, rs, ss)
    print("N=262144 stress: relative to the larger part", et, es, "plain", rel(tau, rt), rel(sig, rs))
    assert et < 1e-5 and es < 1e-5, (et, es)


def test_batch_of_full_size_faults_matches_individual_plans_bitwise():
    from sbiem_inputs import ensemble_members
    pkg = _pkg()
    ws = ensemble_members("ensemble16-N262144")[:2]
    a = [_workload_plan_and_oracle(w, 1)[0] for w in ws]
    b = [_workload_plan_and_oracle(w, 1)[0] for w in ws]
    batch = pkg.Batch(a)
    batch.run(18)
    for p, w in zip(b, ws):
        p.run(w.dt, 18)
    for pa, pb in zip(a, b):
        ga, gb = pa.get_state(), pb.get_state()
        for k in ("slip", "V", "theta", "tau_el", "sigma_el"):
            assert np.array_equal(ga[k], gb[k]), k
    batch.close()


@pytest.mark.parametrize("tile", [512, 64])
def test_tuned_runs_equal_untuned_runs_bitwise(tile):
    """Autotuning replays ordinary steps with several convolution grids and
    launch orders; with the tile fixed (sbiem_set_conv_tile) results do not
    depend on them, so a tuned plan ends where an untuned one run for the
    same number of steps does (plans and batches; tile 64: packed rows,
    whose grids and orders are tuned like the tiles')."""
    pkg = _pkg()
    sc = Scenario(512, 10e3, 0.5 * (10e3 / 512) / CS, rough_10km(512, seed=6), theta_mode="exp",
                  spec=FrictionSpec(overstress=8e6), consistent_V0=True)
    a = make_plan(sc, pkg.SBIEM_FP32CONV)
    b = make_plan(sc, pkg.SBIEM_FP32CONV)
    a.set_conv_tile(tile)
    b.set_conv_tile(tile)
    grid = a.tune(sc.dt, 16)
    assert a.conv_tile() == tile
    assert grid >= 1
    a.run(sc.dt, 37)
    done = a.steps_done()
    assert done > 37
    b.run(sc.dt, done)
    ga, gb = a.get_state(), b.get_state()
    for k in ("slip", "V", "theta", "tau_el", "sigma_el"):
        assert np.array_equal(ga[k], gb[k]), k
    # a batch of two faults against its members stepped alone
    p1, p2 = make_plan(sc, pkg.SBIEM_FP32CONV), make_plan(sc, pkg.SBIEM_FP32CONV)
    p1.set_conv_tile(tile)
    p2.set_conv_tile(tile)
    bt = pkg.Batch([p1, p2])
    bt.tune(16)
    assert p1.conv_tile() == p2.conv_tile() == tile
    n = p1.steps_done()
    assert n == p2.steps_done() > 0
    q = make_plan(sc, pkg.SBIEM_FP32CONV)
    q.set_conv_tile(tile)
    q.run(sc.dt, n)
    g1, gq = p1.get_state(), q.get_state()
    for k in ("slip", "V", "theta", "tau_el", "sigma_el"):
        assert np.array_equal(g1[k], gq[k]), k


def test_tuning_over_tile_shapes():
    """Automatic tuning also tries the 256-, 320-, 512- and 1024-record tiles: the
    plan and the batch keep one of them, and a run on the chosen tile stays
    within the FP32 tolerance of untuned runs (a tile only reorders the FP32
    history sums); a plan set to the chosen tile reproduces the steps after
    tuning bit for bit."""
    pkg = _pkg()
    sc = Scenario(1024, 10e3, 0.5 * (10e3 / 1024) / CS, rough_10km(1024, seed=7), theta_mode="exp",
                  spec=FrictionSpec(overstress=1e6), consistent_V0=True)
    a = make_plan(sc, pkg.SBIEM_FP32CONV)
    a.tune(sc.dt, 16)
    tile = a.conv_tile()
    assert tile in (256, 320, 512, 1024)
    n = a.steps_done()
    b = make_plan(sc, pkg.SBIEM_FP32CONV)
    b.run(sc.dt, n)
    a.run(sc.dt, 40)
    b.run(sc.dt, 40)
    ga, gb = a.get_state(), b.get_state()
    print("tuned tile", tile, "after", n, "tuning steps; tau difference", rel(ga["tau_el"], gb["tau_el"]))
    assert rel(ga["tau_el"], gb["tau_el"]) < 1e-5 and rel(ga["sigma_el"], gb["sigma_el"]) < 1e-5
    # the same tile from the start, then the same steps: bit for bit equal
    c, d = make_plan(sc, pkg.SBIEM_FP32CONV), make_plan(sc, pkg.SBIEM_FP32CONV)
    c.set_conv_tile(tile)
    d.set_conv_tile(tile)
    c.run(sc.dt, 25)
    d.run(sc.dt, 10)
    d.run(sc.dt, 15)
    gc, gd = c.get_state(), d.get_state()
    for k in ("slip", "V", "tau_el", "sigma_el"):
        assert np.array_equal(gc[k], gd[k]), k
    # a batch of two faults
    p1, p2 = make_plan(sc, pkg.SBIEM_FP32CONV), make_plan(sc, pkg.SBIEM_FP32CONV)
    bt = pkg.Batch([p1, p2])
    bt.tune(16)
    assert p1.conv_tile() == p2.conv_tile() in (256, 320, 512, 1024)
    bt.run(20)
    g1, g2 = p1.get_state(), p2.get_state()
    for k in ("slip", "V", "tau_el", "sigma_el"):
        assert np.array_equal(g1[k], g2[k]), k


# ---------------------------------------------------------------- edge cases
@pytest.mark.parametrize("N", [8, 16])
def test_smallest_sizes_match_oracle(N):
    """N = 8 and 16: transforms of P = 2 and 4 points per element class,
    stress path and twenty steps in FP64 against the oracle."""
    from oracle.spectral import curvature
    from oracle.stress import stress_from_history
    from oracle.windows import midpoint_weights
    pkg = _pkg()
    L = 10.0 * N
    dt = 0.5 * (L / N) / CS
    # the rough-fault band (wavelengths 20 dx .. L) is empty at these sizes:
    # two explicit Fourier modes instead
    x = np.arange(N) * (L / N)
    h = 0.4 * np.sin(2 * np.pi * x / L) + 0.15 * np.cos(4 * np.pi * x / L + 0.3)
    hist = _history(N, 60, seed=N)
    p = pkg.Plan(N, L, MU, NU, CS, CP, h)
    tau, sig = p.stress(hist, dt)
    w = midpoint_weights(N, L, CS, CP, dt)
    rt, rs = stress_from_history(hist, dt, L, MU, CS, CP, curvature(h, L), w)
    assert rel(tau, rt) < 1e-10 and rel(sig, rs) < 1e-10, (rel(tau, rt), rel(sig, rs))
    sc = Scenario(N, L, dt, h, theta_mode="exp", spec=FrictionSpec(overstress=3e6),
                  consistent_V0=True)
    q = make_plan(sc, pkg.SBIEM_FP64)
    o = make_oracle(sc)
    q.run(dt, 20)
    o.run(20)
    g = q.get_state()
    for k, ref in (("slip", o.slip), ("V", o.V), ("tau_el", o.tau_el), ("sigma_el", o.sigma_el)):
        assert rel(g[k], ref) < 1e-10, (k, rel(g[k], ref))


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_planar_fault_and_zero_history(precision):
    """h = 0: no normal traction (the packed transform's imaginary part is
    rounding only) and the shear traction of the flat-fault oracle; a zero
    slip history gives zero traction exactly."""
    from oracle.stress import stress_from_history
    from oracle.windows import midpoint_weights
    pkg = _pkg()
    N, L = 512, 5120.0
    dt = 0.5 * (L / N) / CS
    p = pkg.Plan(N, L, MU, NU, CS, CP)
    p.set_precision(pkg.SBIEM_FP64 if precision == "fp64" else pkg.SBIEM_FP32CONV)
    hist = _history(N, 200, seed=3)
    tau, sig = p.stress(hist, dt)
    w = midpoint_weights(N, L, CS, CP, dt)
    rt, _ = stress_from_history(hist, dt, L, MU, CS, CP, np.zeros(N), w)
    tol = 1e-10 if precision == "fp64" else 1e-5
    assert rel(tau, rt) < tol, rel(tau, rt)
    assert np.max(np.abs(sig)) <= (1e-12 if precision == "fp64" else 1e-5) * np.max(np.abs(rt))
    z = np.zeros_like(hist)
    tz, sz = p.stress(z, dt)
    assert not np.any(tz) and not np.any(sz)


def test_stress_at_the_largest_size():
    """N = 2^22, the largest size a plan accepts (FP32 ring of 51 GB, element
    and mode transforms of 2048 points).  A slip held still over the window
    leaves only the static terms, whose closed forms hold at any size
    (sections 2.3 and 2.4 in the static limit): for u = D0 + D cos(k_m x) on
    h = A sin(k_0 x), tau = -mu (1-r) k_m D cos(k_m x) and sigma =
    mu (1-r) A k_0^2 [D0 cos(k_0 x) + D/2 (cos((k_0+k_m) x) + sgn(k_0-k_m)
    cos((k_0-k_m) x))].  The exact weights of every mode are too costly for
    the oracle at this size; the moving case is compared at N = 262144."""
    pkg = _pkg()
    N = 1 << 22
    L = 10.0 * N
    dt = 0.5 * (L / N) / CS
    x = np.arange(N) * (L / N)
    m0, mm, A, D0, D = 3000, 70001, 2.0, 0.7, 0.2
    k0, km = 2 * np.pi * m0 / L, 2 * np.pi * mm / L
    h = A * np.sin(k0 * x)
    u = D0 + D * np.cos(km * x)
    hist = np.repeat(u[None, :], 4, axis=0)
    p = pkg.Plan(N, L, MU, NU, CS, CP, h)
    p.set_precision(pkg.SBIEM_FP32CONV)
    tau, sig = p.stress(hist, dt)
    r = (CS / CP) ** 2
    rt = -MU * (1 - r) * km * D * np.cos(km * x)
    rs = MU * (1 - r) * A * k0 ** 2 * (D0 * np.cos(k0 * x) + 0.5 * D * (
        np.cos((k0 + km) * x) + np.sign(k0 - km) * np.cos((k0 - km) * x)))
    print("N=2^22 static stress:", rel(tau, rt), rel(sig, rs))
    assert rel(tau, rt) < 1e-5 and rel(sig, rs) < 1e-5, (rel(tau, rt), rel(sig, rs))
    p.close()


@pytest.mark.parametrize("N", [4096, 16384, 65536])
def test_stress_fp64_transform_sizes(N):
    """FP64 stress path at the sizes whose element and mode transforms run as
    register wave FFTs (64, 128 and 256 points per class) against the oracle."""
    from oracle.spectral import curvature_fft
    from oracle.stress import stress_from_history
    from oracle.windows import midpoint_weights
    from sbiem_inputs import rough_fault
    pkg = _pkg()
    L = 10.0 * N
    dt = 0.5 * (L / N) / CS
    h = rough_fault(N, L, 3e-3, N)
    nt = 6
    hist = _history(N, nt, seed=N + 1)
    p = pkg.Plan(N, L, MU, NU, CS, CP, h)
    tau, sig = p.stress(hist, dt)
    w = midpoint_weights(N, L, CS, CP, dt, max_lag=nt)
    # the curvature is data here (the library's, rounded from its
    # extended-precision h''): numpy's FFT h'' differs from it by the FP64
    # rounding of the forward transform amplified by k^2 (about 1e-10 at
    # these sizes), which is not part of the time step being compared
    kappa = p.get_curvature()
    assert rel(kappa, curvature_fft(h, L)) < 1e-8
    rt, rs = stress_from_history(hist, dt, L, MU, CS, CP, kappa, w, transform="fft")
    print(f"fp64 stress N={N}:", rel(tau, rt), rel(sig, rs))
    assert rel(tau, rt) < 1e-10 and rel(sig, rs) < 1e-10, (rel(tau, rt), rel(sig, rs))
