"""GPU parity at the full sizes of the measured workloads (256^3, 512^3),
in the launch configuration the benchmark times (default plan, graph replay).

The oracle cannot run these sizes whole, so the checks use values it can
compute: single transform coefficients evaluated one by one, and the
Taylor-Green run of the Re = 1600 case, whose low Fourier modes and energy /
enstrophy history are resolution independent while the cascade is far from
the dealias cutoff (tests/test_oracle_resolution.py) and are stored from a
64^3 oracle run in tests/golden/tg_re1600_n64.npz.
"""
import os

import numpy as np
import pytest

import workloads
from gpu_util import (band_limited_spectrum, box_index, embed_low_modes, embed_on_device, note, radix_plan,
                      to_dev, to_host)
from oracle import spectral

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def tg_ref():
    return np.load(os.path.join(GOLDEN, "tg_re1600_n64.npz"))


def _solver(N, dtype, **kw):
    from paper_1602_03638_amd import Solver
    return Solver(N, 1.0 / 1600, 1e-3, dtype=dtype, **kw)


def _low_mode_error(s, ref, step):
    N = s.N
    uh = to_host(s.get_spectral()) / float(N) ** 3
    got = uh[embed_low_modes(N, ref["kxy"], ref["kz"])]
    want = ref[f"modes_{step}"]
    return float(np.max(np.abs(got - want)) / np.max(np.abs(want)))


def test_tg256_fp64_history_100_steps(tg_ref):
    """256^3 FP64, nu = 1/1600, dt = 1e-3, 100 steps: energy and enstrophy
    after every step and the low modes after 10 and 50 steps."""
    note("tg256 fp64 100 steps")
    s = _solver(256, "f64", diag_every=1)
    s.set_velocity(to_dev(workloads.taylor_green(256), "f64"))
    s.step(10)
    assert _low_mode_error(s, tg_ref, 10) <= 1e-12
    s.step(40)
    assert _low_mode_error(s, tg_ref, 50) <= 1e-12
    s.step(50)
    E, W = s.history()
    assert len(E) == 100
    E_ref, W_ref = tg_ref["energy"][1:], tg_ref["enstrophy"][1:]
    assert np.max(np.abs(np.array(E) - E_ref) / E_ref) <= 1e-12
    assert np.max(np.abs(np.array(W) - W_ref) / W_ref) <= 1e-12


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_tg512_ten_steps(tg_ref, dtype, tol):
    """512^3, 10 steps: low modes, energy and enstrophy against the oracle
    (FP64 to 1e-12, FP32 to 1e-5 relative)."""
    note(f"tg512 {dtype} 10 steps")
    s = _solver(512, dtype)
    s.set_velocity(to_dev(workloads.taylor_green(512), dtype))
    s.step(10)
    E, W = s.diagnostics()
    assert abs(E - tg_ref["energy"][10]) / tg_ref["energy"][10] <= tol
    assert abs(W - tg_ref["enstrophy"][10]) / tg_ref["enstrophy"][10] <= tol
    assert _low_mode_error(s, tg_ref, 10) <= tol
    s.close()


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-13), ("f32", 2e-6)])
def test_forward_512_sampled_modes(dtype, tol):
    """Forward 3D transform of a random 512^3 field: sampled coefficients
    against the definition, evaluated one by one by the oracle."""
    note(f"forward 512 {dtype} sampled")
    N = 512
    u = workloads.random_physical(N, seed=512)
    if dtype == "f32":
        u = u.astype(np.float32).astype(np.float64)
    s = _solver(N, dtype)
    uh = s.forward(to_dev(u, dtype))
    rng = np.random.default_rng(1)
    samples = [(0, 0, 0), (N // 2, N // 2, N // 2), (N - 1, 1, N // 2 - 1)] + \
              [tuple(int(v) for v in rng.integers(0, [N, N, N // 2 + 1])) for _ in range(5)]
    scale = np.sqrt(float(N) ** 3)      # rms size of a coefficient of unit white noise
    for ix, iy, iz in samples:
        got = to_host(uh[:, ix, iy, iz])
        want = spectral.dft3_mode(u, ix, iy, iz)
        assert np.max(np.abs(got - want)) / scale <= tol, (ix, iy, iz)
    s.close()


# Band-limited broadband field: |k_i| <= KB, so u x omega has |k_i| <= 2 KB = 42,
# inside the 2/3-rule mask of 128^3 (3 * 42 < 128) and free of aliasing there.
KB, N_ORACLE = 21, 128


@pytest.fixture(scope="module")
def band_rhs():
    """A band-limited random solenoidal field and its right-hand side from the
    oracle at 128^3 (nu = 0.0137)."""
    uh = band_limited_spectrum(N_ORACLE, seed=421, kb=KB)
    nu = 0.0137
    r = spectral.rhs(uh, nu, spectral.wavenumber_mesh(N_ORACLE), spectral.dealias_mask(N_ORACLE))
    return uh, r, nu


def check_band_rhs(N, dtype, band_rhs, tol, radix=0, **sched):
    """dns_rhs at N^3 of the band-limited field against the oracle's 128^3
    right-hand side: every mode of the box |k_i| <= 2 KB element by element
    (scaled by (N/128)^3), and every mode outside the box (the zero high
    modes, the masked modes and the Nyquist planes) zero to rounding.
    radix != 0: every pass that has a variant of that radix plan at its
    default shape runs it.  Returns the relative L2 error over all stored
    modes."""
    torch = __import__("torch")
    uh, ref, nu = band_rhs
    src = uh if dtype == "f64" else uh.astype(np.complex64).astype(np.complex128)
    if dtype == "f32":
        ref = spectral.rhs(src, nu, spectral.wavenumber_mesh(N_ORACLE), spectral.dealias_mask(N_ORACLE))
    from paper_1602_03638_amd import Solver
    s = Solver(N, nu, 1e-3, dtype=dtype, **sched)
    if radix:
        plan, moved = radix_plan(s, radix)
        assert moved, f"no variant of radix plan {radix} at N={N}"
        s.set_plan_ex(plan)
        note(f"  radix plan {radix} on {', '.join(moved)}")
    dev = embed_on_device(src, N, dtype, KB)
    s.set_spectral(dev)
    del dev
    out = s.rhs()
    s.close()
    scale = (float(N) / N_ORACLE) ** 3
    kb2 = 2 * KB
    bi = box_index(N, kb2, torch)
    got = np.stack([to_host(out[c][bi]) for c in range(3)]) / scale
    want = ref[(slice(None),) + box_index(N_ORACLE, kb2)]
    for c in range(3):
        out[c][bi] = 0
    w_out = float(torch.linalg.vector_norm(out).item()) / scale    # everything outside the box
    del out
    torch.cuda.empty_cache()
    wz = np.full(kb2 + 1, 2.0)
    wz[0] = 1.0
    num = np.sqrt(np.sum(wz * np.abs(got - want) ** 2) + 2 * w_out ** 2)
    den = np.sqrt(np.sum(wz * np.abs(want) ** 2))
    err = float(num / den)
    note(f"  band rhs N={N} {dtype}: rel L2 {err:.2e} (outside box {w_out / den:.1e})")
    assert err <= tol
    return err


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-13), ("f32", 2e-5)])
def test_rhs_512_band_limited_matches_oracle_128(dtype, tol, band_rhs):
    """512^3 right-hand side of a broadband band-limited field, element by
    element against the oracle evaluated at 128^3 (the launch configuration
    of the benchmark: default plan)."""
    note(f"band rhs 512 {dtype}")
    check_band_rhs(512, dtype, band_rhs, tol)


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12), ("f32", 5e-6)])
def test_rhs_512_radix4_plan_matches_oracle_128(dtype, tol, band_rhs):
    """The radix-4 plan (512 = 4 4 4 8, radix plan 2, the one that differs
    from the default at 512) on every pass at the benchmark's size: the same
    element-by-element comparison with the oracle at 128^3."""
    note(f"band rhs 512 {dtype} radix plan 2")
    check_band_rhs(512, dtype, band_rhs, tol, radix=2)


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12), ("f32", 5e-6)])
def test_inverse_512_sampled_points(dtype, tol):
    """dns_inverse of a random (not Hermitian) 512^3 half spectrum: sampled
    physical values against the oracle's point evaluation of the definition
    (which keeps numpy irfftn's treatment of the kz = 0 and N/2 bins),
    relative to the field's rms."""
    note(f"inverse 512 {dtype} sampled points")
    N = 512
    h = workloads.random_half_spectrum(N, seed=5120)
    if dtype == "f32":
        h = h.astype(np.complex64).astype(np.complex128)
    s = _solver(N, dtype)
    u = s.inverse(to_dev(h, dtype))
    s.close()
    rms = float(u.double().pow(2).mean().sqrt().item())
    rng = np.random.default_rng(3)
    pts = [(0, 0, 0), (N - 1, N - 1, N - 1), (1, 2, 3), (N // 2, 7, N // 2 + 1)] + \
          [tuple(int(v) for v in rng.integers(0, N, 3)) for _ in range(4)]
    for i, j, l in pts:
        want = spectral.idft3_point(h, i, j, l)
        got = to_host(u[:, i, j, l])
        assert np.max(np.abs(got - want)) / rms <= tol, (i, j, l, got, want)
    del u
