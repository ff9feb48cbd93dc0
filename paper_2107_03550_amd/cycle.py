"""Seismic-cycle driver (section 6) and the slip/curvature scaling check
(section 5) on top of the C ABI.

``run_cycle`` advances an adaptive plan with ``sbiem_adapt_until``: the
library's step-size control runs the steps; the run stops at each crossing
of the event threshold so that the slip at the start and end of every
seismic event is read exactly there.  This module only orchestrates calls
and keeps the catalogue; every step runs in the library.

``scaling_check`` compares the scaled slip gradient (1/(f du)) d(du)/dx of
``sbiem_slip_scaling`` with -kappa away from the fault's edges, where the
section-5 scaling is expected to hold.

Run ``python -m paper_2107_03550_amd.cycle --help`` for the command line.
"""

from __future__ import annotations

import argparse
import json
import time

import numpy as np

from . import _lib

YEAR = 365.25 * 86400.0


def make_cycle_plan(w, fields, device_precision=None):
    """An adaptive plan for a cycle workload ``w`` with friction ``fields``
    (``sbiem_inputs.friction_fields``): constrained elements set, state at
    t = 0, dt_min = w.dt."""
    p = _lib.Plan(w.N, w.L, w.mu, w.nu, w.cs, w.cp, w.h)
    prec = w.precision if device_precision is None else device_precision
    p.set_precision(_lib.SBIEM_FP64 if prec == "fp64" else _lib.SBIEM_FP32CONV)
    p.set_theta_mode(_lib.SBIEM_THETA_EXP)
    p.set_adaptive(True)
    fr = fields
    p.set_friction(fr["a"], fr["b"], fr["Dc"], fr["V_ref"], fr["f0"], fr["sigma_load"],
                   fr["tau_load"], fr["tau_load_rate"], fr["V_pl"])
    if "constrained" in fr:
        p.set_constrained(fr["constrained"])
    p.set_state(fr["slip0"], fr["V0"], fr["theta0"], 0.0)
    p.set_dt(w.dt)
    return p


def run_cycle(plan, *, eps0, dt_max, t_end, v_event, dt0=None, max_accepted=5_000_000,
              chunk=100_000, free=None, progress=None, max_events=None):
    """Advance ``plan`` to ``t_end`` (or ``max_accepted`` accepted steps, or
    the end of event number ``max_events``).

    Returns a dict: ``t``, ``dt``, ``vmax`` per accepted step (end time,
    step length, maximum slip rate after it); ``events``: one dict per span
    with maximum slip rate above ``v_event`` (t_start, t_end, peak V,
    hypocentre index, slip increment, rupture extent = the share of the free
    elements whose slip increment exceeds 1 % of its maximum); ``attempts``
    by outcome; ``status`` of the last call; ``state`` at the end; wall
    seconds.  ``free``: mask of the elements that may slide (for the extent).
    """
    dt = float(dt0) if dt0 is not None and dt0 > 0 else 1.0
    ts, dts, vms = [], [], []
    counts = dict.fromkeys(_lib.ADAPT_OUTCOMES, 0)
    events = []
    open_ev = None
    accepted = 0
    status = 0
    t0 = time.perf_counter()
    st = plan.get_state()
    if st["V"].max() >= v_event:
        open_ev = dict(t_start=st["t"], slip_start=st["slip"].copy(),
                       hypocentre=int(np.argmax(st["V"])), peak=float(st["V"].max()))
    while accepted < max_accepted and plan.get_state()["t"] < t_end:
        want = min(chunk, max_accepted - accepted)
        status, dt, log, crossed = plan.adapt_until(eps0, dt_max, dt, want, v_event, t_end=t_end,
                                                    log_cap=8 * want + 64)
        for t_a, h, eps, outcome, vmax in log:
            name = _lib.ADAPT_OUTCOMES[int(outcome)]
            counts[name] += 1
            if name in ("accept", "floor"):
                ts.append(t_a + h)
                dts.append(h)
                vms.append(vmax)
                accepted += 1
                if open_ev is not None:
                    open_ev["peak"] = max(open_ev["peak"], float(vmax))
        if progress is not None:
            progress(accepted, ts[-1] if ts else 0.0, len(events))
        if status != 0:
            break
        if crossed:
            st = plan.get_state()
            if open_ev is None:
                open_ev = dict(t_start=st["t"], slip_start=st["slip"].copy(),
                               hypocentre=int(np.argmax(st["V"])), peak=float(st["V"].max()))
            else:
                inc = st["slip"] - open_ev.pop("slip_start")
                mask = np.ones(inc.size, bool) if free is None else np.asarray(free, bool)
                top = inc[mask].max() if mask.any() else 0.0
                open_ev.update(t_end=st["t"], slip=inc,
                               extent=float(np.mean(inc[mask] > 0.01 * top)) if top > 0 else 0.0)
                events.append(open_ev)
                open_ev = None
                if max_events is not None and len(events) >= max_events:
                    break
    wall = time.perf_counter() - t0
    return dict(t=np.array(ts), dt=np.array(dts), vmax=np.array(vms), events=events,
                attempts=counts, status=status, state=plan.get_state(), wall_s=wall,
                accepted=accepted, next_dt=dt)


def interior_mask(free, dx, trim):
    """Free elements at least ``trim`` metres from the free zone's edges."""
    free = np.asarray(free, bool)
    n = int(round(trim / dx))
    keep = free.copy()
    for s in range(1, n + 1):
        keep &= np.roll(free, s) & np.roll(free, -s)
    return keep


def scaling_check(slip, kappa, L, f, keep, slip_floor=0.0):
    """Scaled slip gradient vs -kappa on the elements ``keep``.

    Returns (ratio, -kappa, fit): fit has the least-squares slope of ratio
    on -kappa through the origin, their correlation coefficient and the
    number of elements used."""
    ratio = _lib.slip_scaling(slip, L, f, slip_floor)
    m = np.asarray(keep, bool) & np.isfinite(ratio)
    y, x = ratio[m], -np.asarray(kappa)[m]
    slope = float(np.dot(x, y) / np.dot(x, x)) if m.any() and np.dot(x, x) > 0 else float("nan")
    corr = float(np.corrcoef(x, y)[0, 1]) if m.sum() > 2 else float("nan")
    return ratio, -np.asarray(kappa), dict(slope=slope, corr=corr, n=int(m.sum()))


def main(argv=None):
    from sbiem_inputs import friction_fields, workload

    ap = argparse.ArgumentParser(description="Seismic cycle on a named workload")
    ap.add_argument("--workload", default="sine-cycle-N4096")
    ap.add_argument("--years", type=float, default=None, help="simulated time (default: t_end)")
    ap.add_argument("--max-accepted", type=int, default=5_000_000)
    ap.add_argument("--trim", type=float, default=1000.0,
                    help="metres left out at each edge of the fault for the scaling check")
    ap.add_argument("--out", default=None, help="write the catalogue and final state (.npz)")
    a = ap.parse_args(argv)
    w = workload(a.workload)
    if w.cycle is None:
        raise SystemExit(f"{a.workload} is not a cycle workload")
    fr = friction_fields(w.N, w.L, w.mu, w.cs, w.friction)
    plan = make_cycle_plan(w, fr)
    t_end = w.cycle["t_end"] if a.years is None else a.years * YEAR
    free = ~fr.get("constrained", np.zeros(w.N, bool))

    def progress(acc, t, nev):
        print(f"accepted {acc}  t = {t / YEAR:.3f} yr  events {nev}", flush=True)

    res = run_cycle(plan, eps0=w.cycle["eps0"], dt_max=w.cycle["dt_max"], t_end=t_end,
                    v_event=w.cycle["v_event"], dt0=w.dt, max_accepted=a.max_accepted,
                    chunk=20_000, free=free, progress=progress)
    keep = interior_mask(free, w.dx, a.trim)
    summary = dict(workload=a.workload, status=res["status"], accepted=res["accepted"],
                   attempts=res["attempts"], t_years=res["state"]["t"] / YEAR,
                   wall_s=res["wall_s"], events=[])
    for ev in res["events"]:
        _, _, fit = scaling_check(ev["slip"], plan.get_curvature(), w.L, w.friction.f0, keep)
        summary["events"].append(dict(t_start_yr=ev["t_start"] / YEAR,
                                      duration_s=ev["t_end"] - ev["t_start"],
                                      peak_V=ev["peak"], hypocentre_x=ev["hypocentre"] * w.dx,
                                      max_slip=float(ev["slip"].max()), extent=ev["extent"],
                                      scaling=fit))
    _, _, fit = scaling_check(res["state"]["slip"], plan.get_curvature(), w.L, w.friction.f0, keep)
    summary["final_slip_scaling"] = fit
    print(json.dumps(summary, indent=1))
    if a.out:
        np.savez(a.out, t=res["t"], dt=res["dt"], vmax=res["vmax"],
                 slip=res["state"]["slip"], kappa=plan.get_curvature(),
                 ev_t=np.array([[e["t_start"], e["t_end"]] for e in res["events"]]).reshape(-1, 2),
                 ev_slip=np.array([e["slip"] for e in res["events"]]).reshape(-1, w.N))
    return 0 if res["status"] == 0 else 1


if __name__ == "__main__":
    raise SystemExit(main())
