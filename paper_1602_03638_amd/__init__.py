"""MI355X-native pseudo-spectral Navier-Stokes RK4 step (arXiv:1602.03638).

The solver itself is the HIP library libdns.so (C ABI in include/dns.h);
this package holds its sources (csrc/), its build script (build.py) and a
ctypes binding (binding.py).
"""
from .binding import (  # noqa: F401
    DnsError, Solver, Ensemble, load_library, header_functions, default_opts, state_bytes, LIB_PATH,
    plan_cache_entries, plan_cache_clear, plan_cache_save, plan_cache_load, workspace_bytes, rhs_noalloc, DNS_RK4, DNS_EULER,
    DNS_OK, DNS_E_INVAL, DNS_E_NOMEM, DNS_E_HIP, DNS_E_STATE, DNS_E_NONFINITE, DNS_E_UNSUPPORTED,
    DNS_FP64, DNS_FP32, DNS_TUNE_REPRODUCIBLE, DNS_TUNE_FASTEST,
)
