"""Seeded synthetic inputs for the non-planar spectral BIEM hot path.

This package only *generates inputs*: fault geometries h(x), friction and
loading fields, and the named workload descriptions.  It contains none of the
method's arithmetic (no kernels, windows, curvature, stress or friction
solve), so both the CPU oracle and the HIP library can consume what it makes
without sharing any code with each other.
"""

from .geometry import rough_fault, seamount, sinusoid, element_positions
from .friction import FrictionSpec, friction_fields, TABLE1_CYCLE
from .configs import Workload, workload, ensemble_members, WORKLOAD_NAMES

__all__ = [
    "rough_fault",
    "seamount",
    "sinusoid",
    "TABLE1_CYCLE",
    "element_positions",
    "FrictionSpec",
    "friction_fields",
    "Workload",
    "workload",
    "ensemble_members",
    "WORKLOAD_NAMES",
]
