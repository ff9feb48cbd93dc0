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
    steady = sigma * (spec.f0 + (a - b) * np.log(spec.V_pl / spec.V_ref)) \
        + mu * spec.V_pl / (2.0 * cs)
    tau_load = steady + spec.overstress * np.exp(-(d_n / spec.w_nuc) ** 2)
    return dict(
        a=a, b=b, Dc=spec.Dc, V_ref=spec.V_ref, f0=spec.f0,
        sigma_load=sigma, tau_load=tau_load, tau_load_rate=spec.tau_load_rate,
        V_pl=spec.V_pl,
        slip0=np.zeros(N), V0=np.full(N, spec.V_init),
        theta0=np.full(N, spec.Dc / spec.V_init),
    )
