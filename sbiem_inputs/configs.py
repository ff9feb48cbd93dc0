"""Named synthetic workloads.

Every workload uses the same elastic medium (mu = 30 GPa, nu = 0.25,
c_s = 3464 m/s, c_p = 6000 m/s), the friction of ``FrictionSpec`` and a fixed
time step dt = beta * dx / c_s with beta = 0.5.

=====================  =========================================================
name                   description
=====================  =========================================================
rough-N256-fp64        one rough fault, N = 256, L = 10 km, alpha = 1e-3,
                       seed 0; FP64 everywhere; 2000 steps
seamount-N8192         one fault, N = 8192, L = 80 km, Gaussian seamount
                       A = 50 m, w = 1 km centred at L/2; FP32 convolution
ensemble64             64 rough faults, N drawn from {1024, ..., 16384}
                       (seed 2999), alpha ~ U[1e-3, 1e-2] (seed 2998),
                       geometry seed 2000 + i, dx = 10 m (L = 10 N metres)
rough-N65536           one rough fault, N = 65536, L = 600 km, alpha = 5e-3,
                       seed 3000 (plain and learned-closure forms)
ensemble16-N262144     16 rough faults, N = 262144, L = 2400 km,
                       alpha ~ U[1e-3, 1e-2] (seed 4999), seeds 4000 + i
sine-cycle-N4096       seismic cycle on a sinusoidal fault: N = 4096,
                       L = 40.96 km (dx = 10 m), the central 10.24 km free,
                       h = 80 sin(2 pi (x - L/2) / 5.12 km) m, Table 1
                       parameters (mu = 40 GPa), 0.01 Pa/s shear loading;
                       adaptive steps, dt_min = 0.25 dx / c_s; FP64
=====================  =========================================================

The seismic-cycle workload gives the elastic medium of Table 1 (mu = 40 GPa)
and a ``cycle`` dict: eps0 (error target of the step-size control on ln V
and ln theta), dt_max, v_event (a seismic event is a time span with maximum
slip rate above it), t_end.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .friction import TABLE1_CYCLE, FrictionSpec
from .geometry import rough_fault, seamount, sinusoid

MU = 30e9
NU = 0.25
CS = 3464.0
CP = 6000.0
BETA = 0.5


@dataclass
class Workload:
    name: str
    N: int
    L: float
    h: np.ndarray
    precision: str = "fp32conv"       # "fp64" or "fp32conv"
    steps: int = 2000
    beta: float = BETA
    mu: float = MU
    nu: float = NU
    cs: float = CS
    cp: float = CP
    friction: FrictionSpec = field(default_factory=FrictionSpec)
    cycle: dict | None = None

    @property
    def dx(self) -> float:
        return self.L / self.N

    @property
    def dt(self) -> float:
        return self.beta * self.dx / self.cs


WORKLOAD_NAMES = ("rough-N256-fp64", "seamount-N8192", "ensemble64",
                  "rough-N65536", "ensemble16-N262144", "sine-cycle-N4096")

YEAR = 365.25 * 86400.0


def ensemble_members(name: str) -> list[Workload]:
    """The member faults of an ensemble workload."""
    if name == "ensemble64":
        Ns = np.array([1024, 2048, 4096, 8192, 16384])
        pick = np.random.Generator(np.random.PCG64(2999)).integers(0, Ns.size, size=64)
        alphas = np.random.Generator(np.random.PCG64(2998)).uniform(1e-3, 1e-2, size=64)
        out = []
        for i in range(64):
            N = int(Ns[pick[i]])
            L = 10.0 * N
            out.append(Workload(f"ensemble64[{i}]", N, L,
                                rough_fault(N, L, float(alphas[i]), 2000 + i),
                                precision="fp32conv", steps=20000))
        return out
    if name == "ensemble16-N262144":
        alphas = np.random.Generator(np.random.PCG64(4999)).uniform(1e-3, 1e-2, size=16)
        N, L = 262144, 2400e3
        return [Workload(f"ensemble16-N262144[{i}]", N, L,
                         rough_fault(N, L, float(alphas[i]), 4000 + i),
                         precision="fp32conv", steps=2000) for i in range(16)]
    raise KeyError(name)


def workload(name: str) -> Workload:
    """A single-fault workload by name."""
    if name == "rough-N256-fp64":
        N, L = 256, 10e3
        return Workload(name, N, L, rough_fault(N, L, 1e-3, 0), precision="fp64", steps=2000)
    if name == "seamount-N8192":
        N, L = 8192, 80e3
        return Workload(name, N, L, seamount(N, L, 50.0, 1000.0), precision="fp32conv", steps=2000)
    if name == "rough-N65536":
        N, L = 65536, 600e3
        return Workload(name, N, L, rough_fault(N, L, 5e-3, 3000), precision="fp32conv", steps=2000)
    if name == "sine-cycle-N4096":
        N, L = 4096, 40960.0
        return Workload(name, N, L, sinusoid(N, L, 80.0, 5120.0), precision="fp64", steps=0,
                        beta=0.25, mu=40e9, friction=TABLE1_CYCLE,
                        cycle=dict(eps0=1e-3, dt_max=1e7, v_event=1e-3, t_end=200.0 * YEAR))
    raise KeyError(name)
