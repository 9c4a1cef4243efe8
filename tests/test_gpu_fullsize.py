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
from gpu_util import embed_low_modes, note, to_dev, to_host
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
