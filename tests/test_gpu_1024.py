"""GPU checks at 1024^3, the size of the random isotropic workload (FP32,
nu = 1e-3, dt = 5e-4, seed 1, k0 = 4, E = 0.5).

The oracle cannot hold a 1024^3 field, so the checks use results fixed by
the mathematics at any size, and the oracle at a size it can evaluate:
  * the right-hand side of a band-limited broadband field (|k_i| <= 21) is
    the same at every N >= 128 up to the scale (N/128)^3, so the default
    1024^3 schedule (six-field x pass, long y slices, 64-bit addressing) is
    compared element by element with the oracle at 128^3;
  * the forward transform of a sum of plane waves a cos(k . x + phi) is
    N^3 a e^{i phi} / 2 at k and zero at every other stored mode (closed form
    of the DFT, which pins axis order, sign and normalisation), and the
    inverse transform of that spectrum is the sum of cosines;
  * dns_rhs of the Taylor-Green field equals the exact DFT of its
    closed-form initial tendency (curl, cross product and projection);
  * the random initial field has E = 0.5 and the semi-discrete energy budget
    dE/dt = -2 nu Omega holds over RK4 steps (trapezoid rule);
  * FP32 and FP64 runs from the same spectrum agree in energy to 1e-5.
"""
import math

import numpy as np
import pytest

from gpu_util import note, torch_mod
from test_gpu_fullsize import band_rhs, check_band_rhs  # noqa: F401  (fixture)

pytestmark = pytest.mark.gpu

N = 1024
NU, DT = 1e-3, 5e-4

# (kx, ky, kz, amplitude, phase) per component; 0 < kz < N/2, distinct k
WAVES = [
    [(1, 0, 1, 1.0, 0.3), (-37, 200, 5, 0.25, -1.1)],
    [(0, 3, 2, 0.5, 2.0), (511, -512, 511, 0.125, 0.7)],
    [(-1, -1, 3, 0.75, -0.4), (300, 17, 250, 0.0625, 1.9)],
]


def _plane_waves(torch, dtype):
    """Physical (3, N, N, N) field of the waves above on x_i = 2 pi i / N; the
    phase (k . i mod N) is reduced in integers before the angle is formed."""
    real = torch.float64 if dtype == "f64" else torch.float32
    u = torch.empty((3, N, N, N), dtype=real, device="cuda")
    i = torch.arange(N, device="cuda", dtype=torch.int64)
    for c, waves in enumerate(WAVES):
        acc = torch.zeros((N, N, N), dtype=torch.float64, device="cuda")
        for kx, ky, kz, a, phi in waves:
            m = ((kx * i)[:, None, None] + (ky * i)[None, :, None] + (kz * i)[None, None, :]) % N
            acc += a * torch.cos(m.to(torch.float64) * (2.0 * math.pi / N) + phi)
            del m
        u[c] = acc.to(real)
        del acc
    return u


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-13), ("f32", 2e-6)])
def test_forward_1024_plane_waves(dtype, tol):
    note(f"forward 1024 {dtype} plane waves")
    torch = torch_mod()
    from paper_1602_03638_amd import Solver
    u = _plane_waves(torch, dtype)
    torch.cuda.empty_cache()             # the library allocates outside torch's cache
    s = Solver(N, NU, DT, dtype=dtype)
    uh = s.forward(u)
    s.close()
    del u
    scale = float(N) ** 3
    for c, waves in enumerate(WAVES):
        for kx, ky, kz, a, phi in waves:
            want = scale * a * complex(math.cos(phi), math.sin(phi)) / 2
            got = complex(uh[c, kx % N, ky % N, kz].item())
            assert abs(got - want) / scale <= tol, (c, kx, ky, kz, got, want)
            uh[c, kx % N, ky % N, kz] = 0
    rest = float(uh.abs().max().item()) / scale
    assert rest <= tol, rest
    del uh
    torch.cuda.empty_cache()


def test_random_isotropic_1024_budget_and_precision():
    """Seeded random isotropic field at 1024^3: E0 = 0.5; after each of two
    FP64 RK4 steps (E_{n+1} - E_n) / dt = -nu (Omega_n + Omega_{n+1}) to the
    time-discretisation error; FP32 from the same spectrum agrees in energy and
    enstrophy to 1e-5 relative."""
    note("random isotropic 1024 fp64 budget")
    torch = torch_mod()
    from paper_1602_03638_amd import Solver
    s = Solver(N, NU, DT, dtype="f64")
    s.init_random(1, k0=4.0, energy=0.5)
    E, W = [], []
    e, w = s.diagnostics()
    E.append(e)
    W.append(w)
    assert abs(E[0] - 0.5) <= 1e-12
    uh0 = s.get_spectral()
    for _ in range(2):
        s.step(1)
        e, w = s.diagnostics()
        E.append(e)
        W.append(w)
    s.close()
    for n in range(2):
        lhs = (E[n + 1] - E[n]) / DT
        rhs = -NU * (W[n] + W[n + 1])
        # trapezoid error ~ dt^2 Omega'' / (12 Omega) ~ 1e-7 relative here
        assert abs(lhs - rhs) <= 1e-5 * abs(rhs), (n, lhs, rhs)
    note("random isotropic 1024 fp32 vs fp64")
    s = Solver(N, NU, DT, dtype="f32")
    s.set_spectral(uh0.to(torch.complex64).contiguous())
    del uh0
    torch.cuda.empty_cache()
    s.step(2)
    e32, w32 = s.diagnostics()
    s.close()
    assert abs(e32 - E[2]) / E[2] <= 1e-5
    assert abs(w32 - W[2]) / W[2] <= 1e-5
    assert np.isfinite(e32) and np.isfinite(w32)


@pytest.mark.parametrize("dtype,tol", [("f32", 5e-6), ("f64", 1e-12)])
def test_rhs_1024_band_limited_matches_oracle_128(dtype, tol, band_rhs):
    """1024^3 right-hand side of a broadband band-limited field against the
    oracle at 128^3, element by element over |k_i| <= 42 and zero elsewhere:
    the paths only the 1024^3 default runs (vorticity formed in the x pass,
    16/32 values per y-pass thread, fields beyond 4 GiB)."""
    note(f"band rhs 1024 {dtype}")
    check_band_rhs(N, dtype, band_rhs, tol)
    torch_mod().cuda.empty_cache()


def _trig_modes(terms):
    """Half-spectrum DFT / N^3 of a sum of separable trigonometric terms
    (component, coefficient, (kind, a) per axis), as {(component, kx, ky, kz):
    value} over kz >= 0.  The Fourier coefficients of the factors are
    cos(a x): 1/2 at +-a; sin(a x): -i/2 at +a, +i/2 at -a; 1: 1 at 0."""
    def coeffs(kind, a):
        if a == 0:
            return {0: 1.0}
        return {a: 0.5, -a: 0.5} if kind == "c" else {a: -0.5j, -a: 0.5j}
    modes = {}
    for c, coef, fx, fy, fz in terms:
        for kx, ax in coeffs(*fx).items():
            for ky, ay in coeffs(*fy).items():
                for kz, az in coeffs(*fz).items():
                    if kz >= 0:
                        key = (c, kx, ky, kz)
                        modes[key] = modes.get(key, 0.0) + coef * ax * ay * az
    return modes


# Taylor-Green field u0 = (sin x cos y cos z, -cos x sin y cos z, 0) and the
# closed form of its nonlinear tendency at t = 0 (the form pinned for the
# oracle in oracle_pins.tg_initial_tendency_error): the projected
# -u0.grad u0 - grad p0 = (-sin 2x cos 2z, -sin 2y cos 2z,
# (cos 2x + cos 2y) sin 2z) / 8; the right-hand side adds -nu |k|^2 u_hat.
TG_U = [(0, 1.0, ("s", 1), ("c", 1), ("c", 1)), (1, -1.0, ("c", 1), ("s", 1), ("c", 1))]
TG_N = [(0, -1 / 8, ("s", 2), ("c", 0), ("c", 2)), (1, -1 / 8, ("c", 0), ("s", 2), ("c", 2)),
        (2, 1 / 8, ("c", 2), ("c", 0), ("s", 2)), (2, 1 / 8, ("c", 0), ("c", 2), ("s", 2))]


def _check_sparse(got, modes, n3):
    """Largest deviation of `got` from the sparse spectrum N^3 * modes (every
    other stored mode must be zero), relative to its largest coefficient;
    `got` is overwritten."""
    scale = n3 * max(abs(v) for v in modes.values())
    err = 0.0
    for (c, kx, ky, kz), v in modes.items():
        ix, iy = kx % N, ky % N
        err = max(err, abs(complex(got[c, ix, iy, kz].item()) - n3 * v))
        got[c, ix, iy, kz] = 0
    return err / scale, float(got.abs().max().item()) / scale


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-13), ("f32", 2e-5)])
def test_rhs_1024_taylor_green_closed_form(dtype, tol):
    """dns_init_velocity(Taylor-Green) and dns_rhs at 1024^3 in the default
    schedule, every stored mode against closed forms: the spectrum u_hat
    against the exact DFT of the field, and the nonlinear part
    RHS + nu |k|^2 u_hat (with the context's own u_hat) against the exact DFT
    of the closed-form initial tendency (zero at every other stored mode, the
    Nyquist planes included).  The nonlinear part is compared separately
    because outside the 2/3 mask the right-hand side is -nu |k|^2 u_hat
    alone, which scales the transform's rounding there by up to 3 nu (N/2)^2.
    This pins the curl, the cross product and the projection of the 1024^3
    code by a result fixed by the mathematics.  The bound is a maximum over
    all 1.6e9 stored modes relative to the largest coefficient: the rounding
    of sampled sines and cosines is shared between points a quarter period
    apart (sin(x + pi/2) = cos x), so it concentrates at kx = +-N/4 next to
    the field's own ky, kz (measured 1.2e-14 FP64, 8.6e-6 FP32 there; the
    ratio of the two is that of the precisions)."""
    note(f"1024 {dtype} Taylor-Green closed-form tendency")
    torch = torch_mod()
    from paper_1602_03638_amd import Solver
    nu = 0.0173
    s = Solver(N, nu, DT, dtype=dtype)
    s.init_velocity("taylor_green")
    uh = s.get_spectral()
    got = s.rhs()
    s.close()
    torch.cuda.empty_cache()
    real = torch.float64 if dtype == "f64" else torch.float32
    k = torch.fft.fftfreq(N, 1.0 / N, dtype=torch.float64, device="cuda")
    kz = torch.arange(N // 2 + 1, dtype=torch.float64, device="cuda")
    k2 = ((k * k)[:, None, None] + (k * k)[None, :, None] + (kz * kz)[None, None, :]).to(real)
    for c in range(3):
        got[c] += (nu * k2) * uh[c]     # N_hat = RHS + nu |k|^2 u_hat
    del k2
    n3 = float(N) ** 3
    eu = _check_sparse(uh, _trig_modes(TG_U), n3)
    del uh
    en = _check_sparse(got, _trig_modes(TG_N), n3)
    del got
    torch.cuda.empty_cache()
    note(f"  u_hat: {eu[0]:.2e} at its modes, {eu[1]:.2e} elsewhere; "
         f"nonlinear part: {en[0]:.2e} at its modes, {en[1]:.2e} elsewhere")
    assert max(eu) <= tol and max(en) <= tol


@pytest.mark.parametrize("rs", [1, 2])
def test_rhs_1024_radix_plans_match_oracle_128(rs, band_rhs):
    """The other radix plans at 1024 (1: 1024 = 2 8 8 8, 2: 1024 = 4^5) on
    every pass, FP32: the band-limited right-hand side element by element
    against the oracle at 128^3, to the default plan's tolerance."""
    note(f"band rhs 1024 f32 radix plan {rs}")
    check_band_rhs(N, "f32", band_rhs, 5e-6, radix=rs)
    torch_mod().cuda.empty_cache()


def test_rhs_1024_xcd_grouped_tiles_bitwise(band_rhs):
    """The XCD-grouped x and y passes (the tiles of a 128-byte line on one
    XCD), and the five-field schedule (vorticity combined in the y pass)
    compute the same bits as the default: the right-hand side and one RK4
    step at 1024^3 FP32."""
    note("1024 fp32 xcd grouping bitwise")
    torch = torch_mod()
    from gpu_util import embed_on_device
    from paper_1602_03638_amd import Solver
    uh, _, nu = band_rhs
    outs = []
    for pair in (False, True, "y", "curl_in_y"):
        s = Solver(N, nu, DT, dtype="f32", xcd_pair=bool(pair), curl_in_y=True if pair == "curl_in_y" else None)
        if pair == "y":
            var = s.plan_variants_ex()
            plan = s.plan_ex()
            for p in ("yinv6", "yfwd3"):
                plan[p] = [i for i, d in enumerate(var[p])
                           if d["xcd_pair"] == 1 and d["width"] == 8 and d["radix"] == 0][0]
            s.set_plan_ex(plan)
        sched = s.schedule()
        assert sched["xstage"]["xcd_pair"] == int(bool(pair)) and sched["xrhs_rk4"]["xcd_pair"] == int(bool(pair))
        dev = embed_on_device(uh.astype(np.complex64), N, "f32", 21)
        s.set_spectral(dev)
        r = s.rhs()
        s.set_spectral(dev).step(1)
        del dev
        outs.append((r.cpu(), s.get_spectral().cpu()))
        del r
        s.close()
        torch.cuda.empty_cache()
    for k in (1, 2, 3):
        assert torch.equal(outs[0][0], outs[k][0]), k
        assert torch.equal(outs[0][1], outs[k][1]), k


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-13), ("f32", 2e-6)])
def test_inverse_1024_plane_waves(dtype, tol):
    """dns_inverse of the plane-wave spectrum (N^3 a e^{i phi} / 2 at each k)
    is the sum of cosines a cos(k . x + phi) at every mesh point."""
    note(f"inverse 1024 {dtype} plane waves")
    torch = torch_mod()
    from paper_1602_03638_amd import Solver
    cdt = torch.complex128 if dtype == "f64" else torch.complex64
    uh = torch.zeros((3, N, N, N // 2 + 1), dtype=cdt, device="cuda")
    for c, waves in enumerate(WAVES):
        for kx, ky, kz, a, phi in waves:
            uh[c, kx % N, ky % N, kz] = float(N) ** 3 * a * complex(math.cos(phi), math.sin(phi)) / 2
    torch.cuda.empty_cache()
    s = Solver(N, NU, DT, dtype=dtype)
    u = s.inverse(uh)
    s.close()
    del uh
    torch.cuda.empty_cache()
    want = _plane_waves(torch, dtype)
    amp = sum(abs(w[3]) for w in WAVES[0])
    err = float((u - want).abs().max().item()) / amp
    note(f"  max error {err:.2e}")
    assert err <= tol
    del u, want
    torch.cuda.empty_cache()
