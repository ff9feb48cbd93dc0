"""Friction parameters, loading and initial state of the synthetic workloads.

Rate-and-state friction with the aging law (section "Model and algorithm").
The fields made here are plain inputs:

* a(x): velocity-strengthening outside a central velocity-weakening zone
  (a_vw where |x - L/2| < vw_half_width*L, a_vs elsewhere; a sharp step);
* b, Dc, V_ref, f0: uniform;
* sigma_load(x): uniform effective normal load (compression positive);
* tau_load(x): the steady-state shear traction at the plate rate
  sigma*(f0 + (a - b) ln(V_pl/V_ref)) + mu*V_pl/(2 c_s), plus a Gaussian
  nucleation overstress of amplitude ``overstress`` and width ``w_nuc``
  centred at ``x_nuc`` (default L/2).  The mu*V_pl/(2 c_s) part balances the
  radiation-damping term at the plate rate, so that with no overstress a fault
  sliding uniformly at V_pl is an exact steady state in the backslip frame;
* initial slip 0, slip rate V_init, state theta = Dc / V_init (steady state).

With ``constrained_outside`` the part of the periodic line outside the
velocity-weakening zone is not velocity-strengthening but constrained (a
"constrained" mask: those elements slide at V_pl, i.e. null slip rate when
V_pl = 0, as the fault-benchmark section does outside its fault).  With
V_pl = 0 (no backslip) the steady shear traction is taken at V_init:
sigma*(f0 + (a - b) ln(V_init/V_ref)) + mu*V_init/(2 c_s).
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .geometry import element_positions


@dataclass(frozen=True)
class FrictionSpec:
    a_vw: float = 0.010
    a_vs: float = 0.025
    vw_half_width: float = 0.3      # fraction of L on each side of L/2
    b: float = 0.015
    Dc: float = 1e-3
    V_ref: float = 1e-6
    f0: float = 0.6
    sigma: float = 50e6
    V_pl: float = 1e-9
    V_init: float = 1e-9
    overstress: float = 1e6
    w_nuc: float = 1000.0
    x_nuc: float | None = None      # None: L/2
    tau_load_rate: float = 0.0
    constrained_outside: bool = False


# Table 1 with the seismic-cycle section's loading: a = 0.012, b = 0.015,
# Dc = 1 cm, reference velocity 1e-9 m/s, f0 = 0.6, sigma = 100 MPa; a
# constant shear-traction rate of 0.01 Pa/s, no backslip, no nucleation
# overstress; the 10.24 km fault is the central quarter of the periodic line
# (the sBIEM line is four times the fault length), constrained outside.
TABLE1_CYCLE = FrictionSpec(a_vw=0.012, a_vs=0.012, vw_half_width=0.125, b=0.015, Dc=0.01,
                            V_ref=1e-9, f0=0.6, sigma=100e6, V_pl=0.0, V_init=1e-9,
                            overstress=0.0, tau_load_rate=0.01, constrained_outside=True)


def friction_fields(N: int, L: float, mu: float, cs: float,
                    spec: FrictionSpec = FrictionSpec()) -> dict:
    """Arrays and scalars describing friction, loading and the initial state."""
    x = element_positions(N, L)
    centre = L / 2.0
    d_vw = np.abs(((x - centre + L / 2.0) % L) - L / 2.0)
    a = np.where(d_vw < spec.vw_half_width * L, spec.a_vw, spec.a_vs).astype(np.float64)
    b = np.full(N, spec.b)
    sigma = np.full(N, spec.sigma)
    xn = centre if spec.x_nuc is None else spec.x_nuc
    d_n = ((x - xn + L / 2.0) % L) - L / 2.0
    V_ss = spec.V_pl if spec.V_pl > 0 else spec.V_init
    steady = sigma * (spec.f0 + (a - b) * np.log(V_ss / spec.V_ref)) \
        + mu * V_ss / (2.0 * cs)
    tau_load = steady + spec.overstress * np.exp(-(d_n / spec.w_nuc) ** 2)
    out = dict(
        a=a, b=b, Dc=spec.Dc, V_ref=spec.V_ref, f0=spec.f0,
        sigma_load=sigma, tau_load=tau_load, tau_load_rate=spec.tau_load_rate,
        V_pl=spec.V_pl,
        slip0=np.zeros(N), V0=np.full(N, spec.V_init),
        theta0=np.full(N, spec.Dc / spec.V_init),
    )
    if spec.constrained_outside:
        held = d_vw >= spec.vw_half_width * L
        out["constrained"] = held
        out["V0"] = np.where(held, spec.V_pl, out["V0"])
    return out
