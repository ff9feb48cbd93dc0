"""Shared test scenarios: the same seeded inputs handed to the HIP library
and to the oracle (each side computes everything else on its own)."""

from __future__ import annotations

import os
from dataclasses import dataclass, field

import numpy as np

from sbiem_inputs import FrictionSpec, friction_fields, rough_fault, seamount

MU, NU, CS, CP = 30e9, 0.25, 3464.0, 6000.0
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "kernel_table_L10km_beta05_N256.npz")
DT_10KM = 0.5 * (10e3 / 256) / CS        # the time step of the golden kernel table


@dataclass
class Scenario:
    N: int
    L: float
    dt: float
    h: np.ndarray
    spec: FrictionSpec = field(default_factory=FrictionSpec)
    theta_mode: str = "paper"
    consistent_V0: bool = False


def golden_table():
    from oracle.windows import KernelTable
    z = np.load(GOLDEN)
    return KernelTable(float(z["delta"]), z["CT"], z["CN"])


def fields(sc: Scenario):
    fr = friction_fields(sc.N, sc.L, MU, CS, sc.spec)
    if sc.consistent_V0:
        from oracle.friction import solve_newton
        V0, ok = solve_newton(fr["tau_load"], fr["sigma_load"], fr["theta0"], fr["a"], fr["b"],
                              fr["f0"], fr["V_ref"], fr["Dc"], MU / (2 * CS), fr["V0"])
        assert ok.all()
        fr["V0"] = V0
    return fr


def make_plan(sc: Scenario, precision):
    import paper_2107_03550_amd as pkg
    p = pkg.Plan(sc.N, sc.L, MU, NU, CS, CP, sc.h)
    p.set_precision(precision)
    p.set_theta_mode(pkg.SBIEM_THETA_EXP if sc.theta_mode == "exp" else pkg.SBIEM_THETA_PAPER)
    fr = fields(sc)
    p.set_friction(fr["a"], fr["b"], fr["Dc"], fr["V_ref"], fr["f0"], fr["sigma_load"],
                   fr["tau_load"], fr["tau_load_rate"], fr["V_pl"])
    p.set_state(fr["slip0"], fr["V0"], fr["theta0"], 0.0)
    p.set_dt(sc.dt)
    return p


def make_oracle(sc: Scenario, table=None, kappa=None):
    """The oracle fault of a scenario; ``kappa`` (e.g. the plan's curvature)
    replaces the oracle's own spectral h'' when given, so that a comparison
    measures the time step alone."""
    from oracle.stepper import OracleFault
    return OracleFault(sc.N, sc.L, MU, CS, CP, dt=sc.dt, friction=fields(sc), h=sc.h,
                       kappa=kappa, table=table, theta_mode=sc.theta_mode)


def rel_parts(a, total, static):
    """FP32 comparison norm: ||a - total||_inf over the largest of ||total||,
    ||static|| and ||total - static|| (where the static and dynamic parts
    cancel, FP32 rounding scales with the parts, not with their sum)."""
    total, static = np.asarray(total), np.asarray(static)
    scale = max(np.max(np.abs(total)), np.max(np.abs(static)), np.max(np.abs(total - static)))
    d = np.max(np.abs(np.asarray(a) - total))
    return d / scale if scale > 0 else d


def rel(a, b):
    """Norm-wise relative difference ||a - b||_inf / ||b||_inf."""
    d = np.max(np.abs(np.asarray(a) - np.asarray(b)))
    s = np.max(np.abs(np.asarray(b)))
    return d / s if s > 0 else d


def rough_10km(N, seed=0, alpha=1e-3):
    return rough_fault(N, 10e3, alpha, seed)


def seamount_h(N, L, A=50.0, w=1000.0):
    return seamount(N, L, A, w)
