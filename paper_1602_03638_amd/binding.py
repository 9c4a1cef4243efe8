"""ctypes binding of libdns.so (declared in include/dns.h).

Argument marshalling only: every step of the solver runs in the HIP kernels
of the library.  PyTorch provides device memory and the current stream.
There is no fallback: if libdns.so has not been built, or no GPU is present,
the calls raise.
"""
import ctypes
import os
import re

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB_PATH = os.path.join(PKG, "libdns.so")
HEADER = os.path.join(ROOT, "include", "dns.h")

DNS_OK = 0
DNS_E_INVAL = -1
DNS_E_NOMEM = -2
DNS_E_HIP = -3
DNS_E_STATE = -4
DNS_E_NONFINITE = -5
DNS_E_UNSUPPORTED = -6
DNS_FP64 = 0
DNS_FP32 = 1
DNS_DEALIAS_TEXT = 0
DNS_DEALIAS_APPENDIX = 1
DNS_RK4 = 0
DNS_EULER = 1
INTEGRATORS = {"rk4": DNS_RK4, "euler": DNS_EULER}


class DnsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class dns_opts(ctypes.Structure):
    _fields_ = [("dealias", ctypes.c_int), ("diag_every", ctypes.c_int),
                ("history_cap", ctypes.c_int), ("use_graph", ctypes.c_int), ("autotune", ctypes.c_int),
                ("fuse", ctypes.c_int), ("integrator", ctypes.c_int), ("mfma_dft", ctypes.c_int),
                ("y_elems", ctypes.c_int), ("curl_in_y", ctypes.c_int), ("xcd_pair", ctypes.c_int)]


class dns_variant(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int), ("xcd_pair", ctypes.c_int), ("y_elems", ctypes.c_int),
                ("curl_in_y", ctypes.c_int), ("radix", ctypes.c_int), ("lds_pad", ctypes.c_int)]


DNS_TUNE_REPRODUCIBLE, DNS_TUNE_FASTEST = 0, 1
TUNE_MODES = {"reproducible": DNS_TUNE_REPRODUCIBLE, "fastest": DNS_TUNE_FASTEST}


def _autotune_opt(autotune):
    """opts.autotune for a constructor argument: False, True (reproducible),
    "reproducible" or "fastest"."""
    if autotune is False or autotune is None:
        return 0
    if autotune is True:
        return 1
    return {"reproducible": 1, "fastest": 2}[autotune]


_lib = None


def load_library(path=LIB_PATH):
    """Load libdns.so once.  torch is imported first so that the library
    binds to the HIP runtime torch already loaded (same soname)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_1602_03638_amd.build` "
                           "(there is no CPU fallback)")
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path, mode=ctypes.RTLD_GLOBAL)
    P, I, D, S = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    PP = ctypes.POINTER(ctypes.c_void_p)
    sigs = {
        "dns_default_opts": (None, [ctypes.POINTER(dns_opts)]),
        "dns_state_bytes": (S, [I, I]),
        "dns_create": (I, [I, D, D, I, PP]),
        "dns_create_ex": (I, [I, D, D, I, ctypes.POINTER(dns_opts), P, PP]),
        "dns_create_ws": (I, [I, D, D, I, ctypes.POINTER(dns_opts), P, S, P, PP]),
        "dns_workspace_bytes": (S, [I, I, ctypes.POINTER(dns_opts)]),
        "dns_destroy": (I, [P]),
        "dns_set_velocity": (I, [P, P]),
        "dns_set_spectral": (I, [P, P]),
        "dns_get_spectral": (I, [P, P]),
        "dns_get_velocity": (I, [P, P]),
        "dns_step": (I, [P, I]),
        "dns_rhs": (I, [P, P]),
        "dns_rhs_noalloc": (I, [I, I, D, I, P, P, P]),
        "dns_energy": (I, [P, ctypes.POINTER(D)]),
        "dns_enstrophy": (I, [P, ctypes.POINTER(D)]),
        "dns_diagnostics": (I, [P, ctypes.POINTER(D), ctypes.POINTER(D)]),
        "dns_history": (I, [P, ctypes.POINTER(D), ctypes.POINTER(D), I, ctypes.POINTER(I)]),
        "dns_steps_taken": (I, [P, ctypes.POINTER(ctypes.c_longlong)]),
        "dns_synchronize": (I, [P]),
        "dns_profile_step": (I, [P, I, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_char_p), I,
                                 ctypes.POINTER(I)]),
        "dns_forward": (I, [P, P, P]),
        "dns_inverse": (I, [P, P, P]),
        "dns_init_velocity": (I, [P, I, ctypes.POINTER(D), I]),
        "dns_init_random": (I, [P, ctypes.c_ulonglong, D, D]),
        "dns_autotune": (I, [P, I]),
        "dns_autotune_ex": (I, [P, I, I]),
        "dns_get_plan": (I, [P, ctypes.POINTER(I), I, ctypes.POINTER(I)]),
        "dns_set_plan": (I, [P, ctypes.POINTER(I), I]),
        "dns_plan_variants": (I, [P, I, ctypes.POINTER(I), I, ctypes.POINTER(I)]),
        "dns_plan_cache_entries": (I, []),
        "dns_copy_rows": (I, [P, P, S, I, S, P]),
        "dns_plan_cache_save": (I, [ctypes.c_char_p]),
        "dns_plan_cache_load": (I, [ctypes.c_char_p]),
        "dns_set_schedule": (I, [P, I, I, I]),
        "dns_plan_variants_ex": (I, [P, I, ctypes.POINTER(dns_variant), I, ctypes.POINTER(I)]),
        "dns_get_plan_ex": (I, [P, ctypes.POINTER(I), I, ctypes.POINTER(I)]),
        "dns_set_plan_ex": (I, [P, ctypes.POINTER(I), I]),
        "dns_plan_cache_clear": (I, []),
        "dns_ens_create": (I, [I, ctypes.POINTER(I), ctypes.POINTER(D), ctypes.POINTER(D), I,
                               ctypes.POINTER(dns_opts), P, PP]),
        "dns_ens_destroy": (I, [P]),
        "dns_ens_size": (I, [P, ctypes.POINTER(I), ctypes.POINTER(I)]),
        "dns_ens_set_velocity": (I, [P, I, P]),
        "dns_ens_set_spectral": (I, [P, I, P]),
        "dns_ens_init_random": (I, [P, I, ctypes.c_ulonglong, D, D]),
        "dns_ens_get_spectral": (I, [P, I, P]),
        "dns_ens_step": (I, [P, I, I]),
        "dns_ens_diagnostics": (I, [P, ctypes.POINTER(D), ctypes.POINTER(D)]),
        "dns_ens_synchronize": (I, [P]),
        "dns_ens_last_error": (ctypes.c_char_p, [P]),
        "dns_strerror": (ctypes.c_char_p, [I]),
        "dns_last_error": (ctypes.c_char_p, [P]),
    }
    for name, (res, args) in sigs.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def header_functions(header=HEADER):
    """Names of every function declared in include/dns.h."""
    with open(header) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dns_[a-z_0-9]+)\s*\(", text)))


def _check(status, ctx=None, what=""):
    if status != DNS_OK:
        lib = load_library()
        msg = lib.dns_strerror(status).decode()
        if ctx:
            detail = lib.dns_last_error(ctx).decode()
            if detail:
                msg += ": " + detail
        raise DnsError(status, f"{what}: {msg}" if what else msg)


def default_opts():
    o = dns_opts()
    load_library().dns_default_opts(ctypes.byref(o))
    return o


def state_bytes(N, dtype):
    return int(load_library().dns_state_bytes(int(N), int(dtype)))


def workspace_bytes(N, dtype, **opts):
    """Device bytes a Solver of this size needs (dns_workspace_bytes)."""
    o = default_opts()
    for k, v in opts.items():
        setattr(o, k, int(v))
    return int(load_library().dns_workspace_bytes(int(N), int(dtype), ctypes.byref(o)))


def plan_cache_entries():
    """Number of autotuned plans cached in this process."""
    return int(load_library().dns_plan_cache_entries())


def plan_cache_clear():
    load_library().dns_plan_cache_clear()


def plan_cache_save(path):
    """Write the tuned-plan cache to a JSON file (dns_plan_cache_save)."""
    _check(load_library().dns_plan_cache_save(os.fsencode(path)), None, "dns_plan_cache_save")


def plan_cache_load(path):
    """Add the plans of a cache file to the cache; returns how many it read."""
    n = load_library().dns_plan_cache_load(os.fsencode(path))
    if n < 0:
        _check(n, None, "dns_plan_cache_load")
    return n


def rhs_noalloc(uh, nu, dealias="text", out=None, stream=None):
    """dns_rhs_noalloc: right-hand side of the (3, N, N, N/2+1) CUDA spectrum
    uh (complex128 -> FP64, complex64 -> FP32, N <= 64) with no context and
    no device allocation by the library; `out` (same shape and dtype) is
    allocated by torch when not given.  Enqueued on torch's current stream
    (or `stream`)."""
    import torch
    N = uh.shape[1]
    if (not uh.is_cuda or uh.dtype not in (torch.complex128, torch.complex64) or tuple(uh.shape) != (3, N, N, N // 2 + 1)
            or not uh.is_contiguous()):
        raise ValueError("expected a contiguous CUDA complex tensor of shape (3, N, N, N/2+1)")
    out = torch.empty_like(uh) if out is None else out
    if out.dtype != uh.dtype or out.shape != uh.shape or not out.is_contiguous() or not out.is_cuda:
        raise ValueError("out must match uh")
    if stream is None:
        stream = torch.cuda.current_stream()
    dt = DNS_FP64 if uh.dtype == torch.complex128 else DNS_FP32
    code = {"text": DNS_DEALIAS_TEXT, "appendix": DNS_DEALIAS_APPENDIX}[dealias]
    lib = load_library()
    st = lib.dns_rhs_noalloc(int(N), dt, float(nu), code, ctypes.c_void_p(uh.data_ptr()),
                             ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(stream.cuda_stream))
    if st != DNS_OK:
        raise DnsError(st, "dns_rhs_noalloc: " + lib.dns_strerror(st).decode() + ": " +
                       lib.dns_last_error(None).decode())
    return out


class Solver:
    """One pseudo-spectral DNS context on the current GPU (see include/dns.h).

    dtype: "f64" or "f32"; integrator: "rk4" (default) or "euler"; mfma_dft:
    y passes with the radix-16 stage on FP16 matrix cores (FP32, N >= 64);
    y_elems / curl_in_y / xcd_pair: schedule of the step (dns_set_schedule;
    None = the default for N);
    workspace: None (the library allocates), "torch" (a uint8 tensor from
    torch's allocator) or a contiguous CUDA tensor of at least
    dns_workspace_bytes bytes, 256-byte aligned, kept alive by the Solver.
    Tensors passed in must be contiguous CUDA tensors:
    physical (3, N, N, N) float64/float32, spectral (3, N, N, N/2+1)
    complex128/complex64.  All work is ordered on torch's current stream at
    construction time.
    """

    def __init__(self, N, nu, dt, dtype="f64", dealias="text", diag_every=0, use_graph=True,
                 history_cap=4096, stream=None, autotune=False, fuse=True, integrator="rk4", mfma_dft=False,
                 workspace=None, y_elems=None, curl_in_y=None, xcd_pair=None):
        import torch
        self._torch = torch
        lib = load_library()
        self.N, self.nu, self.dt = int(N), float(nu), float(dt)
        self.dtype = dtype
        self.code = {"f64": DNS_FP64, "f32": DNS_FP32}[dtype]
        self.real = torch.float64 if dtype == "f64" else torch.float32
        self.complex = torch.complex128 if dtype == "f64" else torch.complex64
        o = default_opts()
        o.dealias = {"text": DNS_DEALIAS_TEXT, "appendix": DNS_DEALIAS_APPENDIX}[dealias]
        o.diag_every = int(diag_every)
        o.use_graph = 1 if use_graph else 0
        o.history_cap = int(history_cap)
        o.autotune = _autotune_opt(autotune)
        o.fuse = 1 if fuse else 0
        o.integrator = INTEGRATORS[integrator]
        o.mfma_dft = 1 if mfma_dft else 0
        o.y_elems = 0 if y_elems is None else int(y_elems)
        o.curl_in_y = -1 if curl_in_y is None else int(bool(curl_in_y))
        o.xcd_pair = -1 if xcd_pair is None else int(bool(xcd_pair))
        self.history_cap = int(history_cap)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = ctypes.c_void_p()
        self._ws = None
        if workspace is None:
            _check(lib.dns_create_ex(self.N, self.nu, self.dt, self.code, ctypes.byref(o),
                                     ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)), None, "dns_create_ex")
        else:
            # device memory from torch's allocator: a fresh uint8 tensor of
            # dns_workspace_bytes, or a caller-provided CUDA tensor
            nbytes = int(lib.dns_workspace_bytes(self.N, self.code, ctypes.byref(o)))
            if workspace == "torch":
                workspace = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
            if not workspace.is_cuda or not workspace.is_contiguous():
                raise ValueError("workspace must be a contiguous CUDA tensor")
            self._ws = workspace
            size = workspace.numel() * workspace.element_size()
            _check(lib.dns_create_ws(self.N, self.nu, self.dt, self.code, ctypes.byref(o),
                                     ctypes.c_void_p(workspace.data_ptr()), size,
                                     ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)), None, "dns_create_ws")
        self._h = h

    # -- helpers ----------------------------------------------------------
    @property
    def handle(self):
        if self._h is None or not self._h.value:
            raise RuntimeError("solver is closed")
        return self._h

    def _phys(self, t):
        N = self.N
        if (not t.is_cuda or t.dtype != self.real or tuple(t.shape) != (3, N, N, N)
                or not t.is_contiguous()):
            raise ValueError(f"expected a contiguous CUDA {self.real} tensor of shape (3, {N}, {N}, {N})")
        return ctypes.c_void_p(t.data_ptr())

    def _spec(self, t):
        N = self.N
        if (not t.is_cuda or t.dtype != self.complex or tuple(t.shape) != (3, N, N, N // 2 + 1)
                or not t.is_contiguous()):
            raise ValueError(f"expected a contiguous CUDA {self.complex} tensor of shape "
                             f"(3, {N}, {N}, {N // 2 + 1})")
        return ctypes.c_void_p(t.data_ptr())

    def _empty_phys(self):
        N = self.N
        return self._torch.empty((3, N, N, N), dtype=self.real, device="cuda")

    def _empty_spec(self):
        N = self.N
        return self._torch.empty((3, N, N, N // 2 + 1), dtype=self.complex, device="cuda")

    # -- API ------------------------------------------------------------------
    def set_velocity(self, u):
        _check(load_library().dns_set_velocity(self.handle, self._phys(u)), self.handle, "dns_set_velocity")
        return self

    def set_spectral(self, uh):
        _check(load_library().dns_set_spectral(self.handle, self._spec(uh)), self.handle, "dns_set_spectral")
        return self

    IC_KINDS = {"taylor_green": 0, "taylor_green_2d": 1, "abc": 2, "shear": 3}

    def init_velocity(self, kind="taylor_green", params=()):
        arr = (ctypes.c_double * max(len(params), 1))(*[float(p) for p in params])
        _check(load_library().dns_init_velocity(self.handle, self.IC_KINDS[kind], arr, len(params)), self.handle,
               "dns_init_velocity")
        return self

    def init_random(self, seed, k0=4.0, energy=0.5):
        _check(load_library().dns_init_random(self.handle, int(seed), float(k0), float(energy)), self.handle,
               "dns_init_random")
        return self

    def get_spectral(self, out=None):
        out = self._empty_spec() if out is None else out
        _check(load_library().dns_get_spectral(self.handle, self._spec(out)), self.handle, "dns_get_spectral")
        return out

    def get_velocity(self, out=None):
        out = self._empty_phys() if out is None else out
        _check(load_library().dns_get_velocity(self.handle, self._phys(out)), self.handle, "dns_get_velocity")
        return out

    def forward(self, u, out=None):
        out = self._empty_spec() if out is None else out
        _check(load_library().dns_forward(self.handle, self._phys(u), self._spec(out)), self.handle,
               "dns_forward")
        return out

    def inverse(self, uh, out=None):
        out = self._empty_phys() if out is None else out
        _check(load_library().dns_inverse(self.handle, self._spec(uh), self._phys(out)), self.handle,
               "dns_inverse")
        return out

    def step(self, n=1):
        _check(load_library().dns_step(self.handle, int(n)), self.handle, "dns_step")
        return self

    def rhs(self, out=None):
        out = self._empty_spec() if out is None else out
        _check(load_library().dns_rhs(self.handle, self._spec(out)), self.handle, "dns_rhs")
        return out

    def diagnostics(self):
        E, W = ctypes.c_double(), ctypes.c_double()
        _check(load_library().dns_diagnostics(self.handle, ctypes.byref(E), ctypes.byref(W)), self.handle,
               "dns_diagnostics")
        return E.value, W.value

    def energy(self):
        E = ctypes.c_double()
        _check(load_library().dns_energy(self.handle, ctypes.byref(E)), self.handle, "dns_energy")
        return E.value

    def enstrophy(self):
        W = ctypes.c_double()
        _check(load_library().dns_enstrophy(self.handle, ctypes.byref(W)), self.handle, "dns_enstrophy")
        return W.value

    def history(self):
        cap = self.history_cap
        E = (ctypes.c_double * max(cap, 1))()
        W = (ctypes.c_double * max(cap, 1))()
        n = ctypes.c_int()
        _check(load_library().dns_history(self.handle, E, W, cap, ctypes.byref(n)), self.handle, "dns_history")
        m = min(n.value, cap)
        return list(E[:m]), list(W[:m])

    def steps_taken(self):
        s = ctypes.c_longlong()
        _check(load_library().dns_steps_taken(self.handle, ctypes.byref(s)), self.handle, "dns_steps_taken")
        return s.value

    def synchronize(self):
        _check(load_library().dns_synchronize(self.handle), self.handle, "dns_synchronize")

    def profile_step(self, nsteps=1):
        ms = (ctypes.c_float * 16)()
        names = (ctypes.c_char_p * 16)()
        n = ctypes.c_int()
        _check(load_library().dns_profile_step(self.handle, int(nsteps), ms, names, 16, ctypes.byref(n)),
               self.handle, "dns_profile_step")
        return {names[i].decode(): float(ms[i]) for i in range(n.value) if ms[i] > 0}

    PASSES = ("xinv_curl", "yinv6", "zcross", "yfwd3", "xrhs_rk4", "xstage")

    def autotune(self, reps=3, mode="reproducible"):
        """Time the variants and keep the fastest plan.  mode "reproducible":
        radix plan 0 only (the tuned plan gives the default plan's bits);
        "fastest": the other radix plans too."""
        _check(load_library().dns_autotune_ex(self.handle, int(reps), TUNE_MODES[mode]), self.handle,
               "dns_autotune_ex")
        return self.plan()

    def plan(self):
        w = (ctypes.c_int * len(self.PASSES))()
        n = ctypes.c_int()
        _check(load_library().dns_get_plan(self.handle, w, len(self.PASSES), ctypes.byref(n)), self.handle,
               "dns_get_plan")
        return dict(zip(self.PASSES, list(w)))

    def set_plan(self, widths):
        if isinstance(widths, dict):
            widths = [widths[p] for p in self.PASSES]
        w = (ctypes.c_int * len(self.PASSES))(*[int(x) for x in widths])
        _check(load_library().dns_set_plan(self.handle, w, len(self.PASSES)), self.handle, "dns_set_plan")
        return self

    def set_schedule(self, y_elems=None, curl_in_y=None, xcd_pair=None):
        """dns_set_schedule; None keeps the default for N."""
        _check(load_library().dns_set_schedule(self.handle, 0 if y_elems is None else int(y_elems),
                                                -1 if curl_in_y is None else int(bool(curl_in_y)),
                                                -1 if xcd_pair is None else int(bool(xcd_pair))),
               self.handle, "dns_set_schedule")
        return self

    def plan_variants_ex(self):
        """Every variant of every pass:
        {pass: [dict(width, xcd_pair, y_elems, curl_in_y, radix, lds_pad)]}."""
        out = {}
        for i, name in enumerate(self.PASSES):
            arr = (dns_variant * 32)()
            n = ctypes.c_int()
            _check(load_library().dns_plan_variants_ex(self.handle, i, arr, 32, ctypes.byref(n)), self.handle,
                   "dns_plan_variants_ex")
            out[name] = [dict(width=v.width, xcd_pair=v.xcd_pair, y_elems=v.y_elems, curl_in_y=v.curl_in_y,
                              radix=v.radix, lds_pad=v.lds_pad) for v in arr[: n.value]]
        return out

    def plan_ex(self):
        """Variant index of every pass."""
        w = (ctypes.c_int * len(self.PASSES))()
        n = ctypes.c_int()
        _check(load_library().dns_get_plan_ex(self.handle, w, len(self.PASSES), ctypes.byref(n)), self.handle,
               "dns_get_plan_ex")
        return dict(zip(self.PASSES, list(w)))

    def set_plan_ex(self, variants):
        if isinstance(variants, dict):
            variants = [variants[p] for p in self.PASSES]
        w = (ctypes.c_int * len(self.PASSES))(*[int(x) for x in variants])
        _check(load_library().dns_set_plan_ex(self.handle, w, len(self.PASSES)), self.handle, "dns_set_plan_ex")
        return self

    COUPLED = ("xinv_curl", "yinv6", "xstage")   # passes whose fields depend on the curl placement

    def plan_with(self, p, v, base=None):
        """Variant indices of `base` (default: the current plan) with variant v
        for pass p; where v changes the curl placement, the other coupled
        passes take a variant of that placement (same width and radix plan
        when there is one, else radix plan 0), so that the plan is
        consistent."""
        base = dict(self.plan_ex() if base is None else base)
        var = self.plan_variants_ex()
        base[p] = v
        cy = var[p][v]["curl_in_y"]
        if p in self.COUPLED:
            for q in self.COUPLED:
                if q == p or var[q][base[q]]["curl_in_y"] == cy:
                    continue
                cur = var[q][base[q]]
                cands = [i for i, d in enumerate(var[q]) if d["curl_in_y"] == cy]
                rank = sorted(cands, key=lambda i: (var[q][i]["radix"] != cur["radix"],
                                                    var[q][i]["width"] != cur["width"], var[q][i]["radix"] != 0))
                base[q] = rank[0]
        return base

    def schedule(self):
        """The current plan's descriptors:
        {pass: dict(width, xcd_pair, y_elems, curl_in_y, radix, lds_pad)}."""
        var = self.plan_variants_ex()
        return {p: var[p][i] for p, i in self.plan_ex().items()}

    def plan_variants(self):
        out = {}
        for i, name in enumerate(self.PASSES):
            w = (ctypes.c_int * 8)()
            n = ctypes.c_int()
            _check(load_library().dns_plan_variants(self.handle, i, w, 8, ctypes.byref(n)), self.handle,
                   "dns_plan_variants")
            out[name] = list(w[: n.value])
        return out

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().dns_destroy(self._h)
        self._h = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


DNS_ENS_BATCHED = 0
DNS_ENS_PER_SIM = 1
DNS_ENS_ONE_GRAPH = 2


def _check_ens(status, ens, what):
    if status != DNS_OK:
        lib = load_library()
        msg = lib.dns_strerror(status).decode()
        if ens:
            detail = lib.dns_ens_last_error(ens).decode()
            if detail:
                msg += ": " + detail
        raise DnsError(status, f"{what}: {msg}")


class Ensemble:
    """Independent simulations advanced together (see include/dns.h).

    Ns, nus, dts: per-member grid size, viscosity and time step.  Members with
    equal (N, nu, dt) are batched into one launch per kernel.
    """

    def __init__(self, Ns, nus, dts, dtype="f64", dealias="text", use_graph=True, fuse=True, autotune=False,
                 integrator="rk4", mfma_dft=False, stream=None):
        import torch
        self._torch = torch
        lib = load_library()
        n = len(Ns)
        self.Ns = [int(v) for v in Ns]
        self.dtype = dtype
        self.real = torch.float64 if dtype == "f64" else torch.float32
        self.complex = torch.complex128 if dtype == "f64" else torch.complex64
        o = default_opts()
        o.dealias = {"text": DNS_DEALIAS_TEXT, "appendix": DNS_DEALIAS_APPENDIX}[dealias]
        o.use_graph = 1 if use_graph else 0
        o.fuse = 1 if fuse else 0
        o.autotune = _autotune_opt(autotune)
        o.integrator = INTEGRATORS[integrator]
        o.mfma_dft = 1 if mfma_dft else 0
        if stream is None:
            stream = torch.cuda.current_stream()
        h = ctypes.c_void_p()
        _check_ens(lib.dns_ens_create(n, (ctypes.c_int * n)(*self.Ns), (ctypes.c_double * n)(*map(float, nus)),
                                      (ctypes.c_double * n)(*map(float, dts)), {"f64": DNS_FP64, "f32": DNS_FP32}[dtype],
                                      ctypes.byref(o), ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)),
                   None, "dns_ens_create")
        self._h = h

    @property
    def handle(self):
        if self._h is None or not self._h.value:
            raise RuntimeError("ensemble is closed")
        return self._h

    def __len__(self):
        return len(self.Ns)

    def classes(self):
        n, k = ctypes.c_int(), ctypes.c_int()
        _check_ens(load_library().dns_ens_size(self.handle, ctypes.byref(n), ctypes.byref(k)), self.handle,
                   "dns_ens_size")
        return k.value

    def _spec(self, i, t):
        N = self.Ns[i]
        if (not t.is_cuda or t.dtype != self.complex or tuple(t.shape) != (3, N, N, N // 2 + 1)
                or not t.is_contiguous()):
            raise ValueError(f"expected a contiguous CUDA {self.complex} tensor of shape (3, {N}, {N}, {N // 2 + 1})")
        return ctypes.c_void_p(t.data_ptr())

    def set_velocity(self, i, u):
        N = self.Ns[i]
        if (not u.is_cuda or u.dtype != self.real or tuple(u.shape) != (3, N, N, N) or not u.is_contiguous()):
            raise ValueError(f"expected a contiguous CUDA {self.real} tensor of shape (3, {N}, {N}, {N})")
        _check_ens(load_library().dns_ens_set_velocity(self.handle, int(i), ctypes.c_void_p(u.data_ptr())),
                   self.handle, "dns_ens_set_velocity")
        return self

    def set_spectral(self, i, uh):
        _check_ens(load_library().dns_ens_set_spectral(self.handle, int(i), self._spec(i, uh)), self.handle,
                   "dns_ens_set_spectral")
        return self

    def init_random(self, i, seed, k0=4.0, energy=0.5):
        _check_ens(load_library().dns_ens_init_random(self.handle, int(i), int(seed), float(k0), float(energy)),
                   self.handle, "dns_ens_init_random")
        return self

    def get_spectral(self, i, out=None):
        N = self.Ns[i]
        if out is None:
            out = self._torch.empty((3, N, N, N // 2 + 1), dtype=self.complex, device="cuda")
        _check_ens(load_library().dns_ens_get_spectral(self.handle, int(i), self._spec(i, out)), self.handle,
                   "dns_ens_get_spectral")
        return out

    def step(self, n=1, batched=True, one_graph=False):
        """Advance every member n steps: batched launches replayed as one graph
        per step (default), all n steps in one graph launch (one_graph), or
        per-simulation launches (batched=False)."""
        mode = DNS_ENS_ONE_GRAPH if one_graph else (DNS_ENS_BATCHED if batched else DNS_ENS_PER_SIM)
        _check_ens(load_library().dns_ens_step(self.handle, int(n), mode), self.handle, "dns_ens_step")
        return self

    def diagnostics(self):
        n = len(self.Ns)
        E = (ctypes.c_double * n)()
        W = (ctypes.c_double * n)()
        _check_ens(load_library().dns_ens_diagnostics(self.handle, E, W), self.handle, "dns_ens_diagnostics")
        return list(E), list(W)

    def synchronize(self):
        _check_ens(load_library().dns_ens_synchronize(self.handle), self.handle, "dns_ens_synchronize")

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().dns_ens_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
