"""CPU FP64 oracle for the non-planar spectral BIEM (Romanet & Ozawa, 2021).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package; only the test-suite, the ``smoke()`` check
of ``__graft_entry__.py`` and the ``cpu_baseline`` leg of ``bench.py`` use it.  It
shares no code with the HIP library (``paper_2107_03550_amd``) and imports
nothing from it.

It is a plain, slow, obviously-correct implementation of what the method
computes, written from the paper:

* ``kernels``   - W, psi and the closed-form shear/normal kernels C^T_II and
                  C^N_II (sections 2.3 and 2.4; appendix A), in mpmath at 30
                  digits (``mp``) or in FP64 with scipy (``fp``);
* ``spectral``  - naive O(N^2) DFT with the e^{-ikx} forward sign fixed by the
                  Fourier pairs of appendix B, and the curvature h'';
* ``windows``   - the wavenumber-dependent truncation window T_w(k) and the
                  midpoint convolution weights (section 3.1, time step);
* ``stress``    - the spectral-time stress functional (tau and sigma) of a
                  slip history (section 3.1, eq. for tau^el and sigma_n^el);
* ``friction``  - the rate-and-state momentum balance (eq. momentum) solved by
                  safeguarded Newton on ln V, and a bisection cross-check;
* ``stepper``   - the two-pass predictor-corrector time step (section 3.3);
* ``bruteforce``- a real-space space-time evaluation of the same functional for
                  tiny N (no FFT, no ring bookkeeping);
* ``closure``   - the exact convolution tail that the learned closure stands
                  in for, and an FP64 reference MLP with its gradients.

Readings of points where the paper is silent, garbled or ambiguous are stated
in each function's docstring.
"""
