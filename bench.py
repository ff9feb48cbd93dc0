"""Throughput benchmark of the sBIEM time step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

NAME is one of rough-N256-fp64, seamount-N8192 (default), ensemble64,
rough-N65536, ensemble16-N262144 (ensembles run as one batch).

One "step" is the whole two-pass time step (history convolution, FFTs,
traction assembly, friction solve, commit) of the named workload with its
inputs resident in HBM.  Prints one JSON line with element-steps/s, the
roofline position of the history-convolution kernel (HIP events around its
launches in one step of every 33 of the timed region, the others replayed
from the step graph) and the CPU oracle timed on a bounded sample of the
same workload.
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


def kernel_hash() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def build_plan(w, pkg):
    from sbiem_inputs import friction_fields
    p = pkg.Plan(w.N, w.L, w.mu, w.nu, w.cs, w.cp, w.h)
    p.set_precision(pkg.SBIEM_FP64 if w.precision == "fp64" else pkg.SBIEM_FP32CONV)
    p.set_theta_mode(pkg.SBIEM_THETA_PAPER)
    fr = friction_fields(w.N, w.L, w.mu, w.cs, w.friction)
    p.set_friction(fr["a"], fr["b"], fr["Dc"], fr["V_ref"], fr["f0"], fr["sigma_load"],
                   fr["tau_load"], fr["tau_load_rate"], fr["V_pl"])
    p.set_state(fr["slip0"], fr["V0"], fr["theta0"], 0.0)
    p.set_dt(w.dt)
    return p, fr


def cpu_baseline(w, fr, budget_s: float):
    """The oracle (as it stands) stepping the same workload on host cores."""
    from oracle.stepper import OracleFault
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        threads = 1
    t0 = time.perf_counter()
    o = OracleFault(w.N, w.L, w.mu, w.cs, w.cp, dt=w.dt, friction=fr, h=w.h)
    setup = time.perf_counter() - t0
    steps = 0
    t0 = time.perf_counter()
    while True:
        o.step()
        steps += 1
        el = time.perf_counter() - t0
        if el > budget_s or steps >= 2000:
            break
    return {
        "value": w.N * steps / el, "unit": "element-steps/s", "cores": threads, "kind": "oracle",
        "sample": f"{steps} steps of {w.name} (N={w.N}) from rest, naive O(N^2) DFT, "
                  f"FP64; kernel tables and setup ({setup:.1f} s) excluded",
    }


def train_closure(pkg):
    """Networks of the learned closure, trained on the GPU (untimed) on pairs
    from plain runs of seamount-N8192 and of the ensemble64 members with
    N <= 4096 (2000 steps each, sampled every 50)."""
    from paper_2107_03550_amd.closure_train import collect_pairs, train_networks
    from sbiem_inputs import ensemble_members, workload
    t0 = time.perf_counter()
    sm = workload("seamount-N8192")
    p, _ = build_plan(sm, pkg)
    pairs = collect_pairs([p], sm.dt, 2000, 50)
    small = [m for m in ensemble_members("ensemble64") if m.N <= 4096][:8]
    plans = [build_plan(m, pkg)[0] for m in small]
    more = collect_pairs(plans, small[0].dt, 2000, 50, batch=pkg.Batch(plans))
    pairs = [(np.concatenate([a[0], b[0]]), np.concatenate([a[1], b[1]])) for a, b in zip(pairs, more)]
    pT, pN, lT, lN = train_networks(pairs, steps=3000, batch=2048, lr=2e-3)
    info = {"pairs": [int(len(x)) for x, _ in pairs], "final_loss": [float(lT[-50:].mean()),
            float(lN[-50:].mean())], "target_variance": [float(y.var(0).sum()) for _, y in pairs],
            "seconds": round(time.perf_counter() - t0, 1)}
    return pT, pN, info


def traffic_from_profiles(workload: str, closure: bool, alg_bytes: float):
    """HBM bytes per conv launch from committed rocprofv3 counter summaries,
    if they were taken on the current kernel source and on this very launch
    (same workload, same form, same algorithmic bytes)."""
    tag = workload + ("-closure" if closure else "")
    path = os.path.join(ROOT, "profiles", f"conv_traffic_{tag}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        z = json.load(f)
    if z.get("kernel_sha256_16") != kernel_hash():
        return None
    if z.get("algorithmic_bytes_per_launch") != alg_bytes:
        return None
    return z.get("bytes_per_launch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default="seamount-N8192")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy (torch.neg, MIB MiB read and written, "
                         "10 launches): the known-size kernel that scales the HBM counters")
    ap.add_argument("--closure", action="store_true",
                    help="time the learned-closure form (networks trained first, untimed, on "
                         "plain runs of seamount-N8192 and ensemble64 members)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "ensembles shard by fault and a single fault by wavenumber across GPUs, "
              "which is not built here.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2107_03550_amd as pkg
    from sbiem_inputs import ensemble_members, workload

    if not torch.cuda.is_available():
        print("bench.py: no GPU", file=sys.stderr)
        sys.exit(1)
    stream = torch.cuda.current_stream()
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
    nets = train_closure(pkg) if args.closure else None

    def make_runner(with_closure):
        if args.workload in ENSEMBLES:
            # an ensemble: one batch of independent faults, stepped together
            members = ensemble_members(args.workload)
            plans = []
            for m in members:
                p, _ = build_plan(m, pkg)
                p.set_stream(stream.cuda_stream)
                if with_closure:
                    p.set_closure(nets[0], nets[1], 0.25)
                plans.append(p)
            r = pkg.Batch(plans)
            return r, members, r.run, plans, None, r.tune
        w = workload(args.workload)
        r, fr = build_plan(w, pkg)
        r.set_stream(stream.cuda_stream)
        if with_closure:
            r.set_closure(nets[0], nets[1], 0.25)
        return r, [w], (lambda k: r.run(w.dt, k)), [r], fr, (lambda k: r.tune(w.dt, k))

    runner, members, run, plans, fr, tune = make_runner(args.closure)
    w = members[0]
    n_total = sum(m.N for m in members)

    # warm-up: autotune the convolution grid on ordinary steps (untimed; the
    # results do not depend on it), then the remaining warm-up steps
    n0 = plans[0].steps_done()
    conv_grid = tune(max(16, min(128, args.warmup)))
    tuned_steps = plans[0].steps_done() - n0
    run(max(0, args.warmup - tuned_steps))
    torch.cuda.synchronize()

    # timed region: K steps; one step in every 33 launched directly with its
    # conv launch bracketed by HIP events on the stream the conv kernel is
    # launched on, the others replayed from the step graph
    runner.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    conv_ms, conv_n, conv_bytes = runner.profile()
    runner.set_profiling(False)
    wall = t1 - t0
    value = n_total * args.steps / wall

    # the same K steps replayed through the captured HIP graph (no events)
    torch.cuda.synchronize()
    g0 = time.perf_counter()
    run(args.steps)
    torch.cuda.synchronize()
    g1 = time.perf_counter()
    graph_value = n_total * args.steps / (g1 - g0)

    avg_ms = conv_ms / max(conv_n, 1)
    achieved = conv_bytes / (avg_ms * 1e-3) / 1e9
    roofline = {
        "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic_from_profiles(args.workload, args.closure, conv_bytes),
        "kernel": "k_conv32" if w.precision != "fp64" else "k_conv64", "conv_workgroups": conv_grid,
        "bytes_per_launch": conv_bytes, "avg_launch_us": round(avg_ms * 1e3, 3),
        "launches": conv_n,
    }
    closure_info = None
    if args.closure:
        # the plain form on the same workload (graph replay) and the closure's
        # stress error against it after the same steps from the same state
        plain, _, prun, pplans, _, ptune = make_runner(False)
        m0 = pplans[0].steps_done()
        ptune(max(16, min(128, args.warmup)))
        prun(max(0, args.warmup - (pplans[0].steps_done() - m0)))
        torch.cuda.synchronize()
        q0 = time.perf_counter()
        prun(args.steps)
        torch.cuda.synchronize()
        q1 = time.perf_counter()
        plain_value = n_total * args.steps / (q1 - q0)
        err_tau = err_v = 0.0
        steps_done = plans[0].steps_done()
        prun(steps_done - pplans[0].steps_done())
        torch.cuda.synchronize()
        for pc, pp in zip(plans, pplans):
            gc, gp = pc.get_state(), pp.get_state()
            err_tau = max(err_tau, float(np.max(np.abs(gc["tau_el"] - gp["tau_el"])) /
                                   max(np.max(np.abs(gp["tau_el"])), 1e-300)))
            err_v = max(err_v, float(np.max(np.abs(gc["V"] - gp["V"])) / np.max(np.abs(gp["V"]))))
        closure_info = {"plain_graph_replay_value": plain_value,
                        "speedup_vs_plain": graph_value / plain_value,
                        "tau_el_rel_err_vs_plain": err_tau, "V_rel_err_vs_plain": err_v,
                        "compared_after_steps": steps_done,
                        "training": nets[2]}

    cpu = None
    if not args.no_cpu and args.workload not in ENSEMBLES and w.N <= 16384:
        cpu = cpu_baseline(w, fr, args.cpu_seconds)
    out = {
        "metric": METRIC, "value": value, "unit": "element-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32" if w.precision != "fp64" else "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "N": w.N if len(members) == 1 else
                   sorted({m.N for m in members}), "elements": n_total,
                   "L_m": w.L if len(members) == 1 else "10 N m" if args.workload == "ensemble64"
                   else w.L, "dt_s": w.dt,
                   "precision": "fp32 convolution/FFT, fp64 friction" if w.precision != "fp64"
                   else "fp64", "window": "learned closure (1/4 window)" if args.closure
                   else "full (plain)", "faults": len(members)},
        "graph_replay_value": graph_value,
        "tuning_steps": tuned_steps,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    if closure_info is not None:
        out["closure"] = closure_info
    print(json.dumps(out))


if __name__ == "__main__":
    main()
