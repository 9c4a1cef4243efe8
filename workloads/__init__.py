"""Seeded synthetic inputs shared by the tests, the smoke check and the
benchmark.  Nothing here performs any step of the solver: these functions only
evaluate closed-form initial velocity fields on the physical mesh
x_i = 2*pi*i/N (Mortensen & Langtangen, Sec. 2, eq. realmesh) or draw seeded
random arrays, returning numpy float64 arrays of shape (3, N, N, N) indexed
[component, x, y, z] (or complex half-spectrum arrays for the random
spectral inputs used by transform tests).
"""
from .fields import (  # noqa: F401
    mesh_1d, taylor_green, taylor_green_2d, abc_flow, shear_mode,
    random_physical, random_half_spectrum, CONFIGS,
)
