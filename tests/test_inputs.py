"""Pins of the synthetic input generators against scalars the paper prints."""

import numpy as np
import pytest

from sbiem_inputs import ensemble_members, rough_fault, seamount, workload


@pytest.mark.parametrize("A,printed", [(30.0, 0.026), (100.0, 0.086), (300.0, 0.26)])
def test_seamount_maximum_slope(A, printed):
    # Seamount section: amplitudes 0.03, 0.1, 0.3 km on a 1 km-wide Gaussian
    # give maximum slopes 2.6 %, 8.6 %, 26 %.
    N, L = 1 << 15, 40e3
    h = seamount(N, L, A, 1000.0)
    slope = np.abs(np.diff(h)).max() / (L / N)
    assert abs(slope - printed) <= 0.5 * 10 ** np.floor(np.log10(printed) - 1) + 1e-4


def test_rough_fault_maximum_slope_statistics():
    # Rough-fault section: alpha in {1e-4, 3e-4, 1e-3, 3e-3} with a 200 m
    # minimum wavelength on L = 10.24 km (dx = 10 m) gives maximum slopes
    # {0.0048, 0.014, 0.048, 0.14}, i.e. about 48 alpha for one realisation.
    # The printed ratio must lie inside the spread of our realisations.
    N, L = 1024, 10240.0
    ratios = []
    for seed in range(100):
        h = rough_fault(N, L, 1e-3, seed)
        k = 2 * np.pi * np.fft.rfftfreq(N, L / N)
        slope = np.fft.irfft(1j * k * np.fft.rfft(h), N)
        ratios.append(np.abs(slope).max() / 1e-3)
    lo, hi = np.percentile(ratios, [5, 95])
    for alpha, printed in ((1e-4, 0.0048), (3e-4, 0.014), (1e-3, 0.048), (3e-3, 0.14)):
        assert lo <= printed / alpha <= hi
    # rms slope of a Hurst-1 profile: 2 pi alpha sqrt(2 ln(lambda_max/lambda_min))
    rms = np.mean([np.std(np.fft.irfft(1j * k * np.fft.rfft(rough_fault(N, L, 1e-3, s)), N))
                   for s in range(100)]) / 1e-3
    assert abs(rms / (2 * np.pi * np.sqrt(2 * np.log(L / 200.0))) - 1) < 0.1


def test_table1_nucleation_lengths():
    # Table 1: L_b = mu' Dc/(b sigma) = 355 m and twice the Rubin-Ampuero
    # length (2/pi) mu' Dc b / (sigma (b-a)^2) = 5.659 km with mu' = mu/(1-nu).
    mu_p = 40e9 / (1 - 0.25)
    Lb = mu_p * 1e-2 / (0.015 * 100e6)
    Linf2 = 2 / np.pi * mu_p * 1e-2 * 0.015 / (100e6 * (0.015 - 0.012) ** 2)
    assert abs(Lb - 355) < 1.0 and abs(Linf2 - 5659) < 1.0


def test_workloads_are_deterministic():
    a = workload("rough-N256-fp64")
    b = workload("rough-N256-fp64")
    assert np.array_equal(a.h, b.h) and a.N == 256 and abs(a.dt - 0.5 * (10e3 / 256) / 3464) < 1e-18
    ens = ensemble_members("ensemble64")
    assert len(ens) == 64 and {m.N for m in ens} <= {1024, 2048, 4096, 8192, 16384}
    assert all(abs(m.dx - 10.0) < 1e-12 for m in ens)
