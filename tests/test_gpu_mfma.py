"""The y passes with one radix-16 DFT stage on FP16 matrix cores (split
high/low operands, FP32 accumulation; dns_opts.mfma_dft) against the FP64
oracle, and against the plain FP32 path.

Tolerances: a plain FP32 right-hand side agrees with the oracle to about
1e-6 relative L2 (the FP32 parity tests allow 2e-5); the split products
keep about 22 bits per term, so the matrix-core stage adds an error of the
same order, and the same 2e-5 bound applies.  After 10 RK4 steps the
energy agrees to 1e-5 relative, as for plain FP32.
"""
import numpy as np
import pytest

import workloads
from gpu_util import note, spectral_rel_l2, to_dev, to_host
from oracle import ic, spectral

pytestmark = pytest.mark.gpu


def _solver(N, nu=0.01, dt=0.005, dtype="f32", **kw):
    from paper_1602_03638_amd import Solver
    return Solver(N, nu, dt, dtype=dtype, **kw)


def _rhs_input(N, seed):
    uh = ic.random_isotropic(N, seed, k0=3.0)
    return uh + 0.05 * np.abs(uh).max() * spectral.dft3(workloads.random_physical(N, seed + 1)) / N ** 1.5


@pytest.mark.parametrize("N", [64, 128])
def test_mfma_rhs_against_oracle(N):
    """One right-hand side (inverse y of 6 fields and forward y of 3 through
    the matrix-core stage) on a broadband input including Nyquist planes."""
    note(f"mfma rhs N={N}")
    nu = 0.0137
    uh = _rhs_input(N, seed=60 + N)
    ref = spectral.rhs(uh.astype(np.complex64).astype(np.complex128), nu, spectral.wavenumber_mesh(N),
                       spectral.dealias_mask(N))
    got = to_host(_solver(N, nu=nu, mfma_dft=True).set_spectral(to_dev(uh, "f32")).rhs())
    plain = to_host(_solver(N, nu=nu).set_spectral(to_dev(uh, "f32")).rhs())
    err, err_plain = spectral_rel_l2(got, ref), spectral_rel_l2(plain, ref)
    note(f"  rel L2 vs oracle: mfma {err:.2e}, plain fp32 {err_plain:.2e}")
    assert err <= 2e-5


@pytest.mark.parametrize("N", [64, 128])
def test_mfma_ten_steps_against_oracle(N):
    """10 RK4 steps of a random solenoidal field: energy and enstrophy to
    1e-5, velocity to 1e-5 relative L2 against the FP64 oracle."""
    note(f"mfma 10 steps N={N}")
    nu, dt = 0.01, 0.005
    uh0 = ic.random_isotropic(N, seed=1003)
    orc = spectral.Solver(N, nu, dt).set_spectral(uh0).step(10)
    s = _solver(N, nu, dt, mfma_dft=True).set_spectral(to_dev(uh0, "f32")).step(10)
    E, W = s.diagnostics()
    assert abs(E - orc.energy()) / orc.energy() <= 1e-5
    assert abs(W - orc.enstrophy()) / orc.enstrophy() <= 1e-5
    assert spectral_rel_l2(to_host(s.get_spectral()), orc.uh) <= 1e-5


def test_mfma_fused_unfused_and_ensemble_agree():
    """The matrix-core y pass is deterministic: fused and unfused schedules
    give the same bits, and a batched ensemble member the same bits as a
    single simulation."""
    note("mfma fused/unfused/ensemble")
    from paper_1602_03638_amd import Ensemble
    N, nu, dt = 64, 0.01, 0.005
    uh0 = ic.random_isotropic(N, seed=1004)
    a = _solver(N, nu, dt, mfma_dft=True, fuse=True).set_spectral(to_dev(uh0, "f32")).step(3)
    b = _solver(N, nu, dt, mfma_dft=True, fuse=False).set_spectral(to_dev(uh0, "f32")).step(3)
    ua = to_host(a.get_spectral())
    assert np.array_equal(ua, to_host(b.get_spectral()))
    ens = Ensemble([N, N], [nu, nu], [dt, dt], dtype="f32", mfma_dft=True)
    ens.set_spectral(0, to_dev(uh0, "f32"))
    ens.set_spectral(1, to_dev(ic.random_isotropic(N, seed=1005), "f32"))
    ens.step(3)
    assert np.array_equal(to_host(ens.get_spectral(0)), ua)
    ens.close()


def test_mfma_unsupported_configurations():
    from paper_1602_03638_amd import DnsError
    note("mfma unsupported")
    for N, dtype in ((64, "f64"), (32, "f32")):
        with pytest.raises(DnsError) as e:
            _solver(N, dtype=dtype, mfma_dft=True)
        assert e.value.status == -6        # DNS_E_UNSUPPORTED


def test_mfma_512_against_fp64():
    """At 512^3 a thread's tile rows take several load batches in the stage
    that forms the vorticity (at 64 and 128 one batch holds them all). From a
    seeded random isotropic field, against the FP64 path from the same
    spectrum (FP64 agrees with the oracle to rounding in the parity tests):
    the right-hand side to 2e-5 relative L2, and after two RK4 steps velocity
    to 1e-5, energy and enstrophy to 1e-6."""
    note("mfma 512 vs fp64")
    import torch
    N, nu, dt = 512, 1e-3, 5e-4
    s = _solver(N, nu, dt, dtype="f64")
    s.init_random(7, k0=4.0, energy=0.5)
    uh0 = s.get_spectral().to(torch.complex64).contiguous()
    # the FP64 reference starts from the FP32-rounded spectrum as well
    s.set_spectral(uh0.to(torch.complex128).contiguous())
    r64 = s.rhs()
    s.step(2)
    E64, W64 = s.diagnostics()
    ref = s.get_spectral()
    s.close()
    torch.cuda.empty_cache()
    s = _solver(N, nu, dt, mfma_dft=True).set_spectral(uh0)
    r32 = s.rhs()
    s.step(2)
    E, W = s.diagnostics()
    got = s.get_spectral()
    s.close()
    del uh0
    err_rhs = float(torch.linalg.vector_norm(r32.to(torch.complex128) - r64) / torch.linalg.vector_norm(r64))
    err = float(torch.linalg.vector_norm(got.to(torch.complex128) - ref) / torch.linalg.vector_norm(ref))
    del got, ref, r32, r64
    torch.cuda.empty_cache()
    note(f"  rhs rel L2 {err_rhs:.2e}, velocity {err:.2e}, energy {abs(E - E64) / E64:.2e}, "
         f"enstrophy {abs(W - W64) / W64:.2e}")
    assert err_rhs <= 2e-5
    assert err <= 1e-5
    assert abs(E - E64) / E64 <= 1e-6 and abs(W - W64) / W64 <= 1e-6


def test_mfma_1024_against_plain_fp32():
    """At 1024^3 (16-point DFT on the matrix cores, 64-point Stockham
    sub-transforms, plain six-field inverse y pass), from the same seeded
    random isotropic field: the right-hand side agrees with the plain FP32
    path to 2e-5 relative L2 (the bound of the 64^3 and 128^3 oracle tests),
    and after two RK4 steps velocity, energy and enstrophy agree to 1e-6
    (the paths differ only through dt times the right-hand side)."""
    note("mfma 1024 vs plain fp32")
    import torch
    N, nu, dt = 1024, 1e-3, 5e-4
    out = []
    for mfma in (False, True):
        s = _solver(N, nu, dt, mfma_dft=mfma)
        s.init_random(1, k0=4.0, energy=0.5)
        r = s.rhs()
        s.step(2)
        out.append((r, s.diagnostics(), s.get_spectral()))
        s.close()
        del r
        torch.cuda.empty_cache()
    r0, (E0, W0), u0 = out[0]
    r1, (E1, W1), u1 = out[1]
    err_rhs = float(torch.linalg.vector_norm(r1 - r0) / torch.linalg.vector_norm(r0))
    err_u = float(torch.linalg.vector_norm(u1 - u0) / torch.linalg.vector_norm(u0))
    del out, r0, r1, u0, u1
    torch.cuda.empty_cache()
    note(f"  rhs rel L2 {err_rhs:.2e}, velocity {err_u:.2e}, energy {abs(E1 - E0) / E0:.2e}, "
         f"enstrophy {abs(W1 - W0) / W0:.2e}")
    assert err_rhs <= 2e-5
    assert err_u <= 1e-6
    assert abs(E1 - E0) / E0 <= 1e-6 and abs(W1 - W0) / W0 <= 1e-6
