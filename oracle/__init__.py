"""CPU oracle for one RK4 step of the rotational-form pseudo-spectral
Navier-Stokes solver (Mortensen & Langtangen, arXiv:1602.03638).

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, FP64 statement of
what the GPU path computes.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import it.  The GPU library never
calls into it and it imports nothing from the GPU package; the two share no
code.  Every discrete Fourier transform here is the plain DFT definition
evaluated as dense matrix products (no FFT), with each twiddle angle reduced
modulo the transform length in integers before the angle is formed.

Parity status of each function is stated in its docstring; all functions in
``spectral`` are pinned by ``tests/test_oracle_*.py`` against closed forms,
brute force and the paper's printed worked example.  ``ic.random_isotropic``
is pinned by its invariants and by published SplitMix64 outputs.
"""
from .spectral import (  # noqa: F401
    wavenumbers, wavenumber_mesh, dealias_mask, dft_matrix, dft3, dft3_mode, idft3, idft3_point, curl_hat,
    cross, project, nonlinear_hat, rhs, rk4_step, euler_step, energy, enstrophy, energy_physical,
    divergence_max,
    Solver,
)
