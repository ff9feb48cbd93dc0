"""Throughput benchmark of the sBIEM time step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
                    [--forms plain,closure] [--no-cpu] [--no-tune] [--cycle-years Y]

NAME is one of rough-N256-fp64, seamount-N8192, ensemble64, rough-N65536,
ensemble16-N262144 (default; ensembles run as one batch of faults).

One "step" is the whole two-pass time step (history convolution, FFTs,
traction assembly, friction solve, commit) of every fault of the workload,
with its inputs resident in HBM.  Each form (plain full windows; learned
closure at a quarter of each window) is timed the same way:

  untimed   autotuning of the convolution launch (ordinary steps), W warm-up
            steps, then K steps that capture every launch path the timed run
            takes;
  timed     K steps (16-step graph replays, the remainder launched directly),
            torch.cuda.synchronize() on both sides;
  profile   a separate pass of at least 33 steps, one in 33 launched directly
            with HIP events around its convolution launch on the stream it
            runs on: the convolution's average launch time for the roofline.

The JSON line reports the plain form as `value` (it meets the parity
tolerance against the oracle), the closure form beside it with its speed-up
and its accuracy against the plain form through a rupture, the roofline of
the history convolution, and the CPU oracle on a bounded sample of the same
workload.  A `cycle` object adds the sinusoidal-fault seismic cycle
(sine-cycle-N4096, adaptive steps): wall time for --cycle-years simulated
years, accepted steps per second, its event catalogue, the slip/curvature
scaling of its slip, and the variable-step convolution's roofline during
the first event (a separate evented pass).
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "element-steps/s (stress+friction) at fixed accuracy; plain vs learned-closure, HBM %"
HBM_PEAK_GBS = 8000.0
KERNEL_SRC = os.path.join(ROOT, "paper_2107_03550_amd", "csrc", "kernels.hip")
ENSEMBLES = ("ensemble64", "ensemble16-N262144")
DEFAULT_WORKLOAD = "ensemble16-N262144"


def kernel_hash() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def build_plan(w, pkg, spec=None, theta_exp=False):
    """A plan of workload member ``w`` with its friction (or ``spec``), state
    and time step set; the explicit state update unless ``theta_exp``."""
    from sbiem_inputs import friction_fields
    p = pkg.Plan(w.N, w.L, w.mu, w.nu, w.cs, w.cp, w.h)
    p.set_precision(pkg.SBIEM_FP64 if w.precision == "fp64" else pkg.SBIEM_FP32CONV)
    p.set_theta_mode(pkg.SBIEM_THETA_EXP if theta_exp else pkg.SBIEM_THETA_PAPER)
    fr = friction_fields(w.N, w.L, w.mu, w.cs, spec or w.friction)
    p.set_friction(fr["a"], fr["b"], fr["Dc"], fr["V_ref"], fr["f0"], fr["sigma_load"],
                   fr["tau_load"], fr["tau_load_rate"], fr["V_pl"])
    p.set_state(fr["slip0"], fr["V0"], fr["theta0"], 0.0)
    p.set_dt(w.dt)
    return p, fr


def members_of(name):
    from sbiem_inputs import ensemble_members, workload
    return ensemble_members(name) if name in ENSEMBLES else [workload(name)]


class Form:
    """The faults of a workload in one form (plain, or closed by networks),
    stepped together on one stream."""

    def __init__(self, pkg, name, stream, nets=None, tile=0):
        self.members = members_of(name)
        self.plans = []
        for m in self.members:
            p, _ = build_plan(m, pkg)
            p.set_stream(stream)
            if nets is not None:
                p.set_closure(nets[0], nets[1], 0.25)
            if tile:
                p.set_conv_tile(tile)
            self.plans.append(p)
        self.batch = pkg.Batch(self.plans) if len(self.plans) > 1 else None
        self.dt = self.members[0].dt
        self.n_total = sum(m.N for m in self.members)
        self.handle = self.batch if self.batch is not None else self.plans[0]

    def close(self):
        if self.batch is not None:
            self.batch.close()
        for p in self.plans:
            p.close()

    def run(self, k):
        if k <= 0:
            return
        if self.batch is not None:
            self.batch.run(k)
        else:
            self.plans[0].run(self.dt, k)

    def tune(self, steps_per_trial):
        if self.batch is not None:
            return self.batch.tune(steps_per_trial)
        return self.plans[0].tune(self.dt, steps_per_trial)


def time_form(form, steps, warmup, tune=True):
    """Untimed tuning and warm-up, the timed K steps, then the separate
    profiling pass.  Returns a dict of the measurements."""
    import torch
    out = {}
    n0 = form.plans[0].steps_done()
    if tune and form.members[0].precision != "fp64":
        t0 = time.perf_counter()
        out["conv_workgroups"] = form.tune(16)
        out["tuning_seconds"] = round(time.perf_counter() - t0, 2)
    form.run(max(warmup, 16))
    form.run(steps)                      # every launch path of the timed run, untimed
    torch.cuda.synchronize()
    out["untimed_steps"] = form.plans[0].steps_done() - n0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    form.run(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    out["value"] = form.n_total * steps / wall
    out["ms_per_step"] = wall / steps * 1e3
    # profiling pass (not timed): HIP events around the conv launch of one
    # step in 33, on the conv's stream
    form.handle.set_profiling(True)
    form.run(max(steps, 133))
    torch.cuda.synchronize()
    ms, n, nbytes = form.handle.profile()
    form.handle.set_profiling(False)
    out["conv_ms"] = ms / max(n, 1)
    out["conv_launches"] = n
    out["conv_bytes"] = nbytes
    out["conv_tile"] = form.plans[0].conv_tile()
    return out


CONV32_SHAPES = {64: "k_conv32p", 256: "k_conv32<4,4>", 320: "k_conv32<5,4>", 512: "k_conv32<8,2>", 1024: "k_conv32<16,1>"}


def roofline(m, workload, closure, fp64):
    achieved = m["conv_bytes"] / (m["conv_ms"] * 1e-3) / 1e9
    tile = m.get("conv_tile")
    return {
        "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": traffic_from_profiles(workload, closure, m["conv_bytes"], tile),
        "kernel": "k_conv64" if fp64 else CONV32_SHAPES.get(tile, "k_conv32"),
        "conv_tile": tile, "conv_workgroups": m.get("conv_workgroups"),
        "bytes_per_launch": m["conv_bytes"],
        "avg_launch_us": round(m["conv_ms"] * 1e3, 3), "launches": m["conv_launches"],
    }


def traffic_from_profiles(workload: str, closure: bool, alg_bytes: float, tile=None,
                          prefix: str = "conv_traffic_"):
    """HBM bytes per conv launch from committed rocprofv3 counter summaries,
    if they were taken on the current kernel source and on this very launch
    (same workload, same form, same tile, same algorithmic bytes); prefix
    "var_traffic_" holds those of the variable-step conv."""
    tag = workload + ("-closure" if closure else "")
    names = [f"{prefix}{tag}.json"]
    if tile is not None:
        names.insert(0, f"{prefix}{tag}_tile{tile}.json")
    for name in names:
        path = os.path.join(ROOT, "profiles", name)
        if not os.path.exists(path):
            continue
        with open(path) as f:
            z = json.load(f)
        if z.get("kernel_sha256_16") != kernel_hash():
            continue
        alg = z.get("algorithmic_bytes_per_launch")
        if alg is None or abs(alg - alg_bytes) > 1e-9 * abs(alg_bytes):
            continue
        if tile is not None and z.get("conv_tile", tile) != tile:
            continue
        return z.get("bytes_per_launch")
    return None


# ---------------------------------------------------------------- seismic cycle
CYCLE_WORKLOAD = "sine-cycle-N4096"
PROFILE_YEARS = 3.0


def measure_cycle(pkg, years):
    """The sinusoidal-fault seismic cycle (adaptive steps, FP64) timed over
    `years` of simulated time from the loaded steady state, its event
    catalogue and the section-5 scaling of its slip; then, in a separate
    evented pass over the first PROFILE_YEARS years, the variable-step
    convolution's average launch (algorithmic bytes: the records inside each
    mode's window at each launch) for the roofline."""
    import torch
    from paper_2107_03550_amd.cycle import (YEAR, interior_mask, make_cycle_plan, run_cycle,
                                            scaling_check)
    from sbiem_inputs import friction_fields, workload
    w = workload(CYCLE_WORKLOAD)
    fr = friction_fields(w.N, w.L, w.mu, w.cs, w.friction)
    free = ~fr["constrained"]
    c = w.cycle
    plan = make_cycle_plan(w, fr)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = run_cycle(plan, eps0=c["eps0"], dt_max=c["dt_max"], t_end=years * YEAR,
                    v_event=c["v_event"], dt0=w.dt, free=free, chunk=20000)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    keep = interior_mask(free, w.dx, 1000.0)
    kappa = plan.get_curvature()
    events = []
    for ev in res["events"]:
        _, _, fit = scaling_check(ev["slip"], kappa, w.L, w.friction.f0, keep)
        events.append({"t_start_yr": round(ev["t_start"] / YEAR, 4),
                       "duration_s": round(ev["t_end"] - ev["t_start"], 3),
                       "peak_V": round(ev["peak"], 4), "max_slip_m": round(float(ev["slip"].max()), 4),
                       "extent": round(ev["extent"], 3),
                       "scaling_corr": round(fit["corr"], 3), "scaling_slope": round(fit["slope"], 3)})
    _, _, fin = scaling_check(res["state"]["slip"], kappa, w.L, w.friction.f0, keep)
    t_sim = res["state"]["t"]
    plan.close()

    # evented pass: every variable-step conv launch of the first PROFILE_YEARS
    # simulated years (loading, the first event and its afterslip), the same
    # launches as the committed rocprofv3 summary of
    # `python -m paper_2107_03550_amd.cycle --years 3`
    prof = make_cycle_plan(w, fr)
    prof.set_profiling(True)
    st, dt, _ = prof.adapt(c["eps0"], c["dt_max"], w.dt, 10 ** 7, t_end=PROFILE_YEARS * YEAR,
                           log_cap=16)
    ms, n, b = prof.profile()
    prof.set_profiling(False)
    prof.close()
    conv = None
    if n:
        achieved = b / (ms / n * 1e-3) / 1e9
        conv = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic_from_profiles(CYCLE_WORKLOAD, False, round(b, 1),
                                                 prefix="var_traffic_"),
                "kernel": "k_conv_var<double>", "bytes_per_launch": round(b, 1),
                "avg_launch_us": round(ms / n * 1e3, 3), "launches": n,
                "pass": f"all launches of the first {PROFILE_YEARS:g} simulated years (evented)"}
    acc = res["accepted"]
    return {"workload": CYCLE_WORKLOAD, "N": w.N, "L_m": w.L, "dt_min_s": w.dt,
            "dtype": "f64", "simulated_years": round(t_sim / YEAR, 4), "wall_s": round(wall, 3),
            "accepted_steps": acc, "attempts": res["attempts"],
            "accepted_steps_per_s": round(acc / wall, 1),
            "simulated_years_per_hour": round(t_sim / YEAR / wall * 3600.0, 1),
            "status": res["status"], "events": events,
            "final_slip_scaling": {"corr": round(fin["corr"], 3), "slope": round(fin["slope"], 3),
                                   "elements": fin["n"]},
            "roofline": conv}


# ---------------------------------------------------------------- closure
def train_closure(pkg):
    """Networks of the learned closure, trained on the GPU (untimed) on pairs
    from plain runs through nucleation and rupture of the seamount-N8192
    fault and of the ensemble64 members with N <= 4096 (1 MPa overstress
    raised to 6 MPa over 15 % of the fault, 2000 steps each, sampled every
    50)."""
    from dataclasses import replace
    from paper_2107_03550_amd.closure_train import collect_pairs, train_networks
    from sbiem_inputs import ensemble_members, workload
    t0 = time.perf_counter()
    sm = workload("seamount-N8192")
    spec = replace(sm.friction, overstress=6e6, w_nuc=0.15 * sm.L)
    p, _ = build_plan(sm, pkg, spec, theta_exp=True)
    pairs = collect_pairs([p], sm.dt, 2000, 50)
    small = [m for m in ensemble_members("ensemble64") if m.N <= 4096][:8]
    plans = [build_plan(m, pkg, replace(m.friction, overstress=6e6, w_nuc=0.15 * m.L),
                        theta_exp=True)[0] for m in small]
    more = collect_pairs(plans, small[0].dt, 2000, 50, batch=pkg.Batch(plans))
    pairs = [(np.concatenate([a[0], b[0]]), np.concatenate([a[1], b[1]])) for a, b in zip(pairs, more)]
    pT, pN, lT, lN = train_networks(pairs, steps=3000, batch=2048, lr=2e-3)
    info = {"pairs": [int(len(x)) for x, _ in pairs],
            "final_loss": [float(lT[-50:].mean()), float(lN[-50:].mean())],
            "target_mean_square": [float(np.mean(np.sum(y.astype(np.float64) ** 2, axis=1)))
                                   for _, y in pairs],
            "seconds": round(time.perf_counter() - t0, 1)}
    return pT, pN, info


def closure_accuracy(pkg, nets):
    """The closure's error against the plain full-window run through a
    rupture: a held-out N = 2048 rough fault (10 m elements) nucleating from
    a 6 MPa overstress over 15 % of its length, 6000 steps compared every
    2; the same with zero networks (the constant extrapolation alone)."""
    from sbiem_inputs import FrictionSpec, rough_fault
    from sbiem_inputs.configs import Workload
    N = 2048
    L = 10.0 * N
    w = Workload("held-out-N2048", N, L, rough_fault(N, L, 1e-3, 777),
                 friction=FrictionSpec(overstress=6e6, w_nuc=0.15 * L))
    ref, _ = build_plan(w, pkg, theta_exp=True)
    runs = {}
    zero = np.zeros(pkg.CLOSURE_PARAMS, np.float32)
    for name, pr in (("trained", nets), ("zero", (zero, zero))):
        p, _ = build_plan(w, pkg, theta_exp=True)
        p.set_closure(pr[0], pr[1], 0.25)
        runs[name] = p
    worst = {k: {"tau_el": 0.0, "V": 0.0} for k in runs}
    arrival = {k: np.full(N, -1) for k in ("plain", *runs)}
    failed = {}
    steps, chunk = 6000, 2
    for k in range(1, steps // chunk + 1):
        ref.run(w.dt, chunk)
        g = ref.get_state()
        arrival["plain"][(arrival["plain"] < 0) & (g["V"] > 1e-3)] = k * chunk
        for name, p in runs.items():
            if name in failed:
                continue
            st = p.run_status(w.dt, chunk)
            if st != 0:
                # a physics failure of the closed run (the plain run went on)
                failed[name] = {"step": k * chunk, "status": pkg.lib.sbiem_status_string(st).decode(),
                                "plain_max_V": float(g["V"].max())}
                continue
            h = p.get_state()
            arrival[name][(arrival[name] < 0) & (h["V"] > 1e-3)] = k * chunk
            for key in ("tau_el", "V"):
                e = np.max(np.abs(h[key] - g[key])) / np.max(np.abs(g[key]))
                worst[name][key] = max(worst[name][key], float(e))
    hit = arrival["plain"] >= 0
    span = int(arrival["plain"][hit].max() - arrival["plain"][hit].min()) if hit.any() else 0
    out = {"scenario": f"{w.name}: {steps} steps through nucleation and rupture, cut 1/4; "
                       f"arrival = first step with V >= 1e-3 m/s (2-step resolution), error "
                       f"relative to the rupture's propagation time over the ruptured elements; "
                       f"errors over the steps each closed run completed",
           "ruptured_elements": int(hit.sum()), "propagation_steps": span,
           "plain_max_V": float(ref.get_state()["V"].max())}
    for name in runs:
        a = arrival[name]
        ok = hit & (a >= 0)
        d = np.abs(a[ok] - arrival["plain"][ok]) / max(span, 1)
        out[name] = {"tau_el_rel_err": worst[name]["tau_el"], "V_rel_err": worst[name]["V"],
                     "arrival_rel_err_max": float(d.max()) if d.size else None,
                     "missed_arrivals": int((hit & (a < 0)).sum()),
                     "failed": failed.get(name)}
    return out


# ---------------------------------------------------------------- CPU
def _threads():
    try:
        from threadpoolctl import threadpool_info
        return max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        return 1


def cpu_baseline_fft(w, lags=(4, 12), steps=3):
    """The oracle with numpy's FFT as its transform step (its large-N
    configuration) stepping one fault of the workload.  Full windows are out
    of reach on the host (3.1e8 history entries per N = 262144 fault, about
    30 GB and hours of weight set-up), so the oracle runs with its windows
    cut to ``lags`` lags, each per-step time (transforms, history sums,
    history shift, friction solve) is measured, and the per-step time of the
    full windows is taken from the straight line through the two (time
    against stored history entries)."""
    from oracle.stepper import OracleFault
    from oracle.windows import window_steps
    from sbiem_inputs import friction_fields
    fr = friction_fields(w.N, w.L, w.mu, w.cs, w.friction)
    pts = []
    setup = 0.0
    for lag in lags:
        t0 = time.perf_counter()
        o = OracleFault(w.N, w.L, w.mu, w.cs, w.cp, dt=w.dt, friction=fr, h=w.h,
                        transform="fft", max_lag=lag)
        setup += time.perf_counter() - t0
        t0 = time.perf_counter()
        for _ in range(steps):
            o.step()
        pts.append((int(o.hM.sum()), (time.perf_counter() - t0) / steps))
    (e1, t1), (e2, t2) = pts
    per_entry = (t2 - t1) / (e2 - e1)
    base = t1 - per_entry * e1
    full = int(np.sum(np.maximum(window_steps(w.N, w.L, w.cs, w.dt) - 1, 0)))
    t_full = base + per_entry * full
    return {
        "value": w.N / t_full, "unit": "element-steps/s", "cores": 1, "kind": "oracle",
        "os_cpu_count": os.cpu_count(),
        "sample": (f"one N={w.N} fault of the workload, oracle with numpy FFT (single-threaded "
                   f"numpy), FP64: {steps} steps each with windows cut to {lags[0]} and {lags[1]} "
                   f"lags ({e1} and {e2} history entries: {t1:.3f} s and {t2:.3f} s per step); "
                   f"full windows ({full} entries) by the line through the two: "
                   f"{t_full:.1f} s per step; set-up ({setup:.1f} s) excluded"),
    }


def cpu_baseline_naive(seconds=10.0):
    """The oracle as specified (explicit O(N^2) DFT sums) on the N = 256
    rough-fault FP64 workload, full windows, for about ``seconds``."""
    from oracle.stepper import OracleFault
    from sbiem_inputs import friction_fields, workload
    w = workload("rough-N256-fp64")
    fr = friction_fields(w.N, w.L, w.mu, w.cs, w.friction)
    t0 = time.perf_counter()
    o = OracleFault(w.N, w.L, w.mu, w.cs, w.cp, dt=w.dt, friction=fr, h=w.h)
    setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    n = 0
    while time.perf_counter() - t0 < seconds and n < w.steps:
        o.step()
        n += 1
    el = time.perf_counter() - t0
    return {"value": w.N * n / el, "unit": "element-steps/s", "cores": _threads(),
            "kind": "oracle", "os_cpu_count": os.cpu_count(),
            "sample": f"{n} steps of rough-N256-fp64 (N=256, full windows), explicit DFT sums, "
                      f"FP64; set-up ({setup:.1f} s) excluded"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD)
    ap.add_argument("--forms", default="plain,closure",
                    help="comma list of plain and closure (closure: networks trained first, "
                         "untimed)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the closure's accuracy run through a rupture")
    ap.add_argument("--conv-tile", type=int, default=0, choices=(0, 64, 256, 320, 512, 1024),
                    help="fix the FP32 conv tile (records); 0: autotuned with the grid")
    ap.add_argument("--cycle-years", type=float, default=35.0,
                    help="simulated years of the sinusoidal-fault cycle measured beside the "
                         "fixed-step forms (0: skip)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy (torch.neg, MIB MiB read and written, "
                         "10 launches): the known-size kernel that scales the HBM counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "ensembles shard by fault and a single fault by wavenumber across GPUs, "
              "which is not built here.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2107_03550_amd as pkg

    if not torch.cuda.is_available():
        print("bench.py: no GPU", file=sys.stderr)
        sys.exit(1)
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.randn(n, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(10):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration": {"bytes_read": 4 * n, "bytes_written": 4 * n,
                                               "launches": 10, "kernel": "torch.neg (elementwise)"}}))
        return
    forms = [f for f in args.forms.split(",") if f]
    stream = torch.cuda.current_stream().cuda_stream
    nets = None
    if "closure" in forms:
        log("training the closure networks (untimed)")
        nets = train_closure(pkg)
    results = {}
    for f in forms:
        log(f"building the {f} form of {args.workload}")
        form = Form(pkg, args.workload, stream, nets[:2] if f == "closure" else None,
                    tile=args.conv_tile)
        log(f"timing the {f} form")
        results[f] = time_form(form, args.steps, args.warmup, tune=not args.no_tune)
        results[f]["n_total"] = form.n_total
        w = form.members[0]
        n_members = len(form.members)
        form.close()
        torch.cuda.synchronize()
    fp64 = w.precision == "fp64"
    first = forms[0]
    m = results[first]
    out = {
        "metric": METRIC, "value": m["value"], "unit": "element-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": m["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if fp64 else "f32", "data": "synthetic",
        "config": {"workload": args.workload,
                   "N": w.N if n_members == 1 else sorted({x.N for x in members_of(args.workload)}),
                   "elements": m["n_total"], "faults": n_members, "L_m": w.L, "dt_s": w.dt,
                   "precision": "fp64" if fp64 else "fp32 convolution/FFT, fp64 friction",
                   "window": "full (plain)" if first == "plain" else "learned closure (1/4)"},
        "roofline": roofline(m, args.workload, first == "closure", fp64),
        "timing": {"tuning_seconds": m.get("tuning_seconds"), "untimed_steps": m["untimed_steps"],
                   "profile_pass": f"{m['conv_launches']} evented conv launches in a separate pass"},
    }
    if "closure" in results and first != "closure":
        c = results["closure"]
        out["closure"] = {
            "value": c["value"], "ms_per_step": c["ms_per_step"],
            "speedup_vs_plain": c["value"] / m["value"],
            "roofline": roofline(c, args.workload, True, fp64),
            "training": nets[2],
        }
        if not args.no_accuracy:
            log("closure accuracy through a rupture")
            out["closure"]["accuracy"] = closure_accuracy(pkg, nets[:2])
    if args.cycle_years > 0:
        log(f"seismic cycle: {args.cycle_years} simulated years of {CYCLE_WORKLOAD}")
        out["cycle"] = measure_cycle(pkg, args.cycle_years)
    if not args.no_cpu:
        log("CPU oracle baselines")
        out["cpu_baseline"] = cpu_baseline_fft(members_of(args.workload)[0]) \
            if w.N >= 8192 else cpu_baseline_naive()
        if w.N >= 8192:
            out["cpu_baseline_naive"] = cpu_baseline_naive()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
