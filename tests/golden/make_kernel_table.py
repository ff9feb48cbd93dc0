"""Write the 30-digit kernel table used by the FP64 parity tests.

Calls only the oracle.  Every FP64 test on a 10 km fault with the time step
of the N = 256 rough-fault workload (dt = 0.5 * (10 km / 256) / c_s) shares
the kernel arguments T_p = p * pi * c_s * dt / L = p * pi / 512, so one table
of C^T_II and C^N_II at p = 0..P serves all of them (mode |n| and lag j use
p = |n| (2j + 1)).

Usage: python tests/golden/make_kernel_table.py   (about 2 minutes on 8 cores)
"""

import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.kernels import kernel_table_mp  # noqa: E402

CS, CP = 3464.0, 6000.0
L = 10e3
N_REF = 256
BETA = 0.5
P_MAX = 34000
OUT = os.path.join(HERE, "kernel_table_L10km_beta05_N256.npz")


def main():
    dt = BETA * (L / N_REF) / CS
    CT, CN = kernel_table_mp(repr(np.pi / 512), P_MAX, CS, CP)
    np.savez_compressed(OUT, CT=CT, CN=CN, delta=np.pi / 512, cs=CS, cp=CP, L=L, dt=dt,
                        p_max=P_MAX)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
