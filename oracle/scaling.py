"""Slip/curvature scaling of section 5 (test infrastructure: only tests/,
the smoke check and the benchmark's CPU baseline use this package).

Section 5 states that in the small-slope in-plane setting the scaled slip
gradient (1/(f du)) d(du)/dy equals -kappa away from the fault's edges.
Its diagnostic on a discrete slip profile is read here as the second-order
centred difference on the periodic element grid x_i = i L/N (the
along-fault distance is x to first order in the slope):

    r_i = (du_{i+1} - du_{i-1}) / (2 dx f du_i),   dx = L/N, indices mod N,

undefined (NaN) where |du_i| <= a slip floor.
"""

from __future__ import annotations

import math

import numpy as np


def scaled_slip_gradient(slip, L, f, slip_floor=0.0):
    """r_i of the module docstring, one element at a time."""
    u = [float(x) for x in slip]
    N = len(u)
    dx = L / N
    out = np.empty(N)
    for i in range(N):
        if abs(u[i]) <= slip_floor:
            out[i] = math.nan
            continue
        du = (u[(i + 1) % N] - u[(i - 1) % N]) / (2.0 * dx)
        out[i] = du / (f * u[i])
    return out


def scaling_slip(h_slope, f, c=1.0):
    """The slip the scaling law predicts for a fault of slope h'(x):
    d ln(du)/dx = -f kappa = -f h'' integrates to du = c exp(-f h')."""
    return c * np.exp(-f * np.asarray(h_slope, dtype=np.float64))
