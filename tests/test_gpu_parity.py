"""GPU parity of the HIP path against the CPU oracle, through the C ABI.

FP64 transforms and right-hand sides agree with the oracle to rounding
(relative L2 <= 1e-13); after 10 RK4 steps of the 32^3 Taylor-Green case
the velocity agrees to relative L2 <= 1e-12 and the energy and enstrophy to
1e-12 relative; FP32 runs agree in energy to 1e-5 relative.
"""
import json
import os

import numpy as np
import pytest

import workloads
from gpu_util import note, radix_plan, rel_l2, spectral_rel_l2, to_dev, to_host
from oracle import ic, spectral

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
TOL_F64 = 1e-13      # one transform or one RHS evaluation, relative L2
TOL_F32 = 2e-6
TOL_STEP10 = 1e-12   # velocity after 10 FP64 RK4 steps, relative L2


def _solver(N, nu=0.01, dt=0.01, dtype="f64", **kw):
    from paper_1602_03638_amd import Solver
    return Solver(N, nu, dt, dtype=dtype, **kw)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("N", [8, 16, 32, 64, 128])
def test_forward_transform(N, dtype):
    note(f"forward N={N} {dtype}")
    u = workloads.random_physical(N, seed=100 + N)
    s = _solver(N, dtype=dtype)
    got = to_host(s.forward(to_dev(u, dtype)))
    ref = spectral.dft3(u)
    assert rel_l2(got, ref) <= (TOL_F64 if dtype == "f64" else TOL_F32)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("N", [8, 16, 32, 64, 128])
def test_inverse_transform_non_hermitian_input(N, dtype):
    """The inverse real transform ignores Im of the kz = 0 and N/2 bins."""
    note(f"inverse N={N} {dtype}")
    h = workloads.random_half_spectrum(N, seed=200 + N)
    s = _solver(N, dtype=dtype)
    got = to_host(s.inverse(to_dev(h, dtype)))
    ref = spectral.idft3(h)
    assert rel_l2(got, ref) <= (TOL_F64 if dtype == "f64" else TOL_F32)


@pytest.mark.parametrize("N", [16, 64])
def test_set_velocity_equals_forward_and_spectral_roundtrip(N):
    note(f"set/get N={N}")
    u = workloads.random_physical(N, seed=7)
    s = _solver(N)
    du = to_dev(u, "f64")
    a = to_host(s.set_velocity(du).get_spectral())
    b = to_host(s.forward(du))
    assert np.array_equal(a, b)
    h = workloads.random_half_spectrum(N, seed=8)
    back = to_host(s.set_spectral(to_dev(h, "f64")).get_spectral())
    assert np.array_equal(back, h)
    v = to_host(s.set_velocity(du).get_velocity())
    assert rel_l2(v, u) <= TOL_F64


def _rhs_input(N, seed):
    """Random solenoidal field plus broadband noise (all modes, including
    the Nyquist planes and modes outside the dealias mask)."""
    uh = ic.random_isotropic(N, seed, k0=3.0)
    return uh + 0.05 * np.abs(uh).max() * spectral.dft3(workloads.random_physical(N, seed + 1)) / N ** 1.5


@pytest.mark.parametrize("dealias", ["text", "appendix"])
@pytest.mark.parametrize("N", [8, 16, 32, 64])
def test_rhs_matches_oracle(N, dealias):
    note(f"rhs N={N} {dealias}")
    nu = 0.0137
    uh = _rhs_input(N, seed=30 + N)
    s = _solver(N, nu=nu, dealias=dealias)
    got = to_host(s.set_spectral(to_dev(uh, "f64")).rhs())
    ref = spectral.rhs(uh, nu, spectral.wavenumber_mesh(N), spectral.dealias_mask(N, dealias))
    assert spectral_rel_l2(got, ref) <= TOL_F64


@pytest.fixture(scope="module")
def rhs_input_256():
    return _rhs_input(256, seed=296)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("N", [128, 256])
def test_rhs_matches_oracle_at_larger_sizes(N, dtype, rhs_input_256):
    """Broadband right-hand side against the oracle where the stage passes
    change form: 128^3 uses plain global accesses, 256^3 streaming ones; both
    form the vorticity in the inverse y pass from five x-pass fields, with
    multi-tile y and x passes and ragged Nyquist-plane workgroups."""
    note(f"rhs N={N} {dtype}")
    nu = 0.0137
    uh = rhs_input_256 if N == 256 else _rhs_input(N, seed=40 + N)
    s = _solver(N, nu=nu, dtype=dtype)
    got = to_host(s.set_spectral(to_dev(uh, dtype)).rhs())
    s.close()
    src = uh if dtype == "f64" else uh.astype(np.complex64).astype(np.complex128)
    ref = spectral.rhs(src, nu, spectral.wavenumber_mesh(N), spectral.dealias_mask(N))
    err = spectral_rel_l2(got, ref)
    note(f"  rel L2 {err:.2e}")
    assert err <= (TOL_F64 if dtype == "f64" else 2e-5)


@pytest.mark.parametrize("N", [16, 32])
def test_rhs_fp32(N):
    note(f"rhs fp32 N={N}")
    nu = 0.0137
    uh = _rhs_input(N, seed=50 + N)
    s = _solver(N, nu=nu, dtype="f32")
    got = to_host(s.set_spectral(to_dev(uh, "f32")).rhs())
    ref = spectral.rhs(uh.astype(np.complex64).astype(np.complex128), nu, spectral.wavenumber_mesh(N),
                       spectral.dealias_mask(N))
    assert spectral_rel_l2(got, ref) <= 2e-5


@pytest.mark.parametrize("use_graph", [True, False])
def test_taylor_green_32_ten_steps(use_graph):
    """Taylor-Green 32^3 FP64, nu = 0.01, dt = 0.01, 10 RK4 steps."""
    note(f"tg32 10 steps graph={use_graph}")
    N, nu, dt = 32, 0.01, 0.01
    u0 = workloads.taylor_green(N)
    orc = spectral.Solver(N, nu, dt).set_velocity(u0).step(10)
    s = _solver(N, nu, dt, use_graph=use_graph)
    s.set_velocity(to_dev(u0, "f64")).step(10)
    u = to_host(s.get_velocity())
    assert rel_l2(u, orc.get_velocity()) <= TOL_STEP10
    uh = to_host(s.get_spectral())
    assert spectral_rel_l2(uh, orc.uh) <= TOL_STEP10
    E, W = s.diagnostics()
    assert abs(E - orc.energy()) / orc.energy() <= 1e-12
    assert abs(W - orc.enstrophy()) / orc.enstrophy() <= 1e-12


def test_random_isotropic_steps_fp64():
    """A broadband nonlinear flow (random solenoidal IC), 5 steps, 32^3."""
    note("iso32 5 steps")
    N, nu, dt = 32, 0.01, 0.005
    uh0 = ic.random_isotropic(N, seed=1000)
    orc = spectral.Solver(N, nu, dt).set_spectral(uh0).step(5)
    s = _solver(N, nu, dt).set_spectral(to_dev(uh0, "f64")).step(5)
    assert spectral_rel_l2(to_host(s.get_spectral()), orc.uh) <= TOL_STEP10


def test_history_every_step():
    note("history tg32")
    N, nu, dt = 32, 0.01, 0.01
    u0 = workloads.taylor_green(N)
    E_ref, W_ref = [], []
    spectral.Solver(N, nu, dt).set_velocity(u0).step(
        10, callback=lambda o: (E_ref.append(o.energy()), W_ref.append(o.enstrophy())))
    s = _solver(N, nu, dt, diag_every=1).set_velocity(to_dev(u0, "f64")).step(10)
    E, W = s.history()
    assert len(E) == 10
    assert np.max(np.abs(np.array(E) - E_ref) / np.array(E_ref)) <= 1e-12
    assert np.max(np.abs(np.array(W) - W_ref) / np.array(W_ref)) <= 1e-12


def test_appendix_worked_example_on_gpu():
    """The paper's Appendix run (N = 128, FP64, 10 steps): printed energy."""
    note("appendix tg128")
    with open(os.path.join(GOLDEN, "appendix_tg128.json")) as f:
        g = json.load(f)
    N = g["N"]
    s = _solver(N, g["nu"], g["dt"], dealias=g["dealias"])
    s.set_velocity(to_dev(workloads.taylor_green(N), "f64")).step(g["steps"])
    u = to_host(s.get_velocity())
    E_phys = 0.5 * np.sum(u * u) / N ** 3
    assert abs(E_phys - g["energy_printed"]) <= 5e-13
    assert abs(s.energy() - g["energy_printed"]) <= 5e-13


@pytest.mark.parametrize("N", [32, 64])
def test_fp32_energy_error(N):
    note(f"fp32 tg N={N}")
    nu, dt = 0.01, 0.01
    u0 = workloads.taylor_green(N)
    orc = spectral.Solver(N, nu, dt).set_velocity(u0).step(10)
    s = _solver(N, nu, dt, dtype="f32").set_velocity(to_dev(u0, "f32")).step(10)
    E, W = s.diagnostics()
    assert abs(E - orc.energy()) / orc.energy() <= 1e-5
    assert abs(W - orc.enstrophy()) / orc.enstrophy() <= 1e-5
    assert rel_l2(to_host(s.get_velocity()), orc.get_velocity()) <= 1e-5


def test_deterministic_and_resumable():
    note("determinism/resume")
    N, nu, dt = 32, 0.01, 0.005
    uh0 = ic.random_isotropic(N, seed=1001)
    a = to_host(_solver(N, nu, dt).set_spectral(to_dev(uh0, "f64")).step(6).get_spectral())
    b = to_host(_solver(N, nu, dt).set_spectral(to_dev(uh0, "f64")).step(6).get_spectral())
    assert np.array_equal(a, b)
    s1 = _solver(N, nu, dt).set_spectral(to_dev(uh0, "f64")).step(3)
    mid = s1.get_spectral()
    c = to_host(_solver(N, nu, dt).set_spectral(mid).step(3).get_spectral())
    assert np.array_equal(a, c)


def test_state_errors():
    from paper_1602_03638_amd import DNS_E_STATE, DnsError
    note("state errors")
    s = _solver(16)
    with pytest.raises(DnsError) as e:
        s.step(1)
    assert e.value.status == DNS_E_STATE
    with pytest.raises(DnsError):
        s.energy()
    with pytest.raises(ValueError):
        s.set_velocity(to_dev(workloads.random_physical(8, 1), "f64"))


def test_nonfinite_energy_reported():
    from paper_1602_03638_amd import DNS_E_NONFINITE, DnsError
    note("nonfinite")
    h = workloads.random_half_spectrum(16, seed=3)
    h[0, 1, 1, 1] = np.nan
    s = _solver(16).set_spectral(to_dev(h, "f64"))
    with pytest.raises(DnsError) as e:
        s.energy()
    assert e.value.status == DNS_E_NONFINITE


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("N", [8, 16, 32, 64])
def test_every_plan_variant_is_bitwise_identical(N, dtype):
    """Variants of radix plan 0 change how lines share a workgroup, which
    workgroup takes a tile, how many values a y-pass thread holds, which
    kernel combines the vorticity and the z pass's shared-memory padding,
    never the arithmetic: every such variant of every pass gives identical
    bits, and so does the autotuner's choice in reproducible mode.  Variants
    of the other radix plans (same transforms, other rounding) agree to
    rounding after two RK4 steps."""
    note(f"plan variants N={N} {dtype}")
    uh0 = ic.random_isotropic(N, seed=77)
    s = _solver(N, 0.01, 0.005, dtype=dtype)
    base = s.plan_ex()
    var = s.plan_variants_ex()
    ref = to_host(s.set_spectral(to_dev(uh0, dtype)).step(2).get_spectral())
    for p, vs in var.items():
        for v in range(len(vs)):
            s.set_plan_ex(s.plan_with(p, v, base))
            got = to_host(s.set_spectral(to_dev(uh0, dtype)).step(2).get_spectral())
            if vs[v]["radix"] == 0:
                assert np.array_equal(got, ref), (p, vs[v])
            else:
                assert spectral_rel_l2(got, ref) <= (TOL_F64 if dtype == "f64" else TOL_F32), (p, vs[v])
    tuned = s.autotune()
    assert all(d["radix"] == 0 for d in s.schedule().values()), tuned
    got = to_host(s.set_spectral(to_dev(uh0, dtype)).step(2).get_spectral())
    assert np.array_equal(got, ref), tuned
    s.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("N", [16, 32, 128])
@pytest.mark.parametrize("rs", [1, 2])
def test_radix_plans_match_oracle(N, dtype, rs):
    """The other radix plans (radix-2/4 stage first; radix-4 stages) compute
    the same discrete transforms: with every pass on plan rs, the broadband
    right-hand side agrees with the oracle element by element (relative L2)
    and the transforms' round trip restores the field.  A plan that equals
    an earlier one for this N has no variants (nothing to test)."""
    note(f"radix plan {rs} N={N} {dtype}")
    nu = 0.0137
    uh = _rhs_input(N, seed=90 + N + rs)
    s = _solver(N, nu=nu, dtype=dtype)
    plan, moved = radix_plan(s, rs)
    l = int(np.log2(N))
    distinct = (rs == 1 and l % 3 != 0) or (rs == 2 and l not in (3, 5))
    assert bool(moved) == distinct, (moved, distinct)
    if not moved:
        s.close()
        pytest.skip(f"radix plan {rs} is an earlier plan at N={N}")
    assert set(moved) == set(s.PASSES), moved
    s.set_plan_ex(plan)
    got = to_host(s.set_spectral(to_dev(uh, dtype)).rhs())
    src = uh if dtype == "f64" else uh.astype(np.complex64).astype(np.complex128)
    ref = spectral.rhs(src, nu, spectral.wavenumber_mesh(N), spectral.dealias_mask(N))
    err = spectral_rel_l2(got, ref)
    note(f"  rel L2 {err:.2e}")
    assert err <= (TOL_F64 if dtype == "f64" else 2e-5)
    s.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_fastest_mode_tuning(dtype):
    """The fastest mode times the variants of every radix plan; its plan
    (whatever it chose) keeps the velocity within rounding of the default
    plan's after two RK4 steps, and the reproducible mode never chooses a
    radix plan other than 0."""
    N = 128
    note(f"fastest-mode tuning N={N} {dtype}")
    uh0 = ic.random_isotropic(N, seed=81)
    d = _solver(N, 0.01, 0.005, dtype=dtype)
    ref = to_host(d.set_spectral(to_dev(uh0, dtype)).step(2).get_spectral())
    d.autotune(mode="reproducible")
    assert all(v["radix"] == 0 for v in d.schedule().values())
    d.close()
    s = _solver(N, 0.01, 0.005, dtype=dtype)
    s.autotune(mode="fastest")
    note(f"  fastest plan {s.schedule()}")
    got = to_host(s.set_spectral(to_dev(uh0, dtype)).step(2).get_spectral())
    assert spectral_rel_l2(got, ref) <= (TOL_F64 if dtype == "f64" else TOL_F32)
    s.close()


def _long_y(dtype):
    """The schedule of the 1024^3 default: six-field x pass (vorticity formed
    in the x pass) and 16 (FP64) / 32 (FP32) values per y-pass thread."""
    return dict(y_elems=16 if dtype == "f64" else 32, curl_in_y=False)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("N", [64, 128])
def test_rhs_with_1024_schedule_matches_oracle(N, dtype):
    """The code the 1024^3 default runs (six-field x pass with the curl
    combinations of the Sec. 3.1 Curl listing formed there; long y slices with
    twiddles in shared memory), selected at a size the oracle evaluates:
    broadband right-hand side element by element, then two fused RK4 steps
    bitwise equal to the default schedule."""
    note(f"rhs 1024-schedule N={N} {dtype}")
    nu = 0.0137
    uh = _rhs_input(N, seed=60 + N)
    s = _solver(N, nu=nu, dtype=dtype, **_long_y(dtype))
    sched = s.schedule()
    assert sched["xinv_curl"]["curl_in_y"] == 0 and sched["xstage"]["curl_in_y"] == 0
    assert sched["yinv6"]["y_elems"] == _long_y(dtype)["y_elems"]
    assert sched["yfwd3"]["y_elems"] == _long_y(dtype)["y_elems"]
    got = to_host(s.set_spectral(to_dev(uh, dtype)).rhs())
    src = uh if dtype == "f64" else uh.astype(np.complex64).astype(np.complex128)
    ref = spectral.rhs(src, nu, spectral.wavenumber_mesh(N), spectral.dealias_mask(N))
    err = spectral_rel_l2(got, ref)
    note(f"  rel L2 {err:.2e}")
    assert err <= (TOL_F64 if dtype == "f64" else 2e-5)
    a = to_host(s.set_spectral(to_dev(uh, dtype)).step(2).get_spectral())
    d = _solver(N, nu=nu, dtype=dtype)
    b = to_host(d.set_spectral(to_dev(uh, dtype)).step(2).get_spectral())
    assert np.array_equal(a, b)
    for x in (s, d):
        x.close()


def test_schedule_errors():
    """Schedules the library does not provide are refused, the plan is left
    as it was, and inconsistent explicit plans are rejected."""
    from paper_1602_03638_amd import DNS_E_INVAL, DNS_E_UNSUPPORTED, DnsError
    note("schedule errors")
    s = _solver(32)
    before = s.plan_ex()
    small = _solver(16)
    with pytest.raises(DnsError) as e:
        small.set_schedule(y_elems=32, curl_in_y=False)  # 32 values per thread: lines of at least 32
    assert e.value.status == DNS_E_UNSUPPORTED
    small.close()
    with pytest.raises(DnsError) as e:
        s.set_schedule(xcd_pair=True)                    # no 64-byte rows at 32^3
    assert e.value.status == DNS_E_UNSUPPORTED
    assert s.plan_ex() == before
    var = s.plan_variants_ex()
    plan = dict(before)
    plan["xinv_curl"] = [i for i, d in enumerate(var["xinv_curl"]) if d["curl_in_y"] == 0][0]
    with pytest.raises(DnsError) as e:
        s.set_plan_ex(plan)
    assert e.value.status == DNS_E_INVAL
    s.set_schedule(curl_in_y=False)
    assert s.schedule()["yinv6"]["curl_in_y"] == 0
    s.set_schedule(y_elems=16, curl_in_y=True)           # the combining inverse pass keeps 8
    sched = s.schedule()
    assert sched["yinv6"]["y_elems"] == 8 and sched["yfwd3"]["y_elems"] == 16
    s.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("N", [16, 64])
def test_fused_schedule_matches_unfused_bitwise(N, dtype):
    """Fusing each stage's RHS pass with the next stage's inverse x pass
    changes where values live, not the arithmetic."""
    note(f"fused vs unfused N={N} {dtype}")
    uh0 = ic.random_isotropic(N, seed=78)
    a = _solver(N, 0.01, 0.005, dtype=dtype, fuse=True).set_spectral(to_dev(uh0, dtype))
    b = _solver(N, 0.01, 0.005, dtype=dtype, fuse=False).set_spectral(to_dev(uh0, dtype))
    a.step(2)
    b.step(2)
    assert np.array_equal(to_host(a.get_spectral()), to_host(b.get_spectral()))
    # get_velocity reuses the work space: the next step must rebuild it
    va, vb = to_host(a.get_velocity()), to_host(b.get_velocity())
    assert np.array_equal(va, vb)
    a.step(3)
    b.step(3)
    assert np.array_equal(to_host(a.get_spectral()), to_host(b.get_spectral()))
    assert a.diagnostics() == b.diagnostics()


@pytest.mark.parametrize("N", [16, 32])
def test_forward_euler_against_oracle(N):
    """Forward Euler (Sec. 3.1 main loop, u_hat += RHS dt), 10 steps of the
    Taylor-Green field and of a random solenoidal field, FP64: velocity to
    1e-12 relative L2 and the per-step energy history to 1e-12."""
    note(f"euler N={N}")
    nu, dt = 0.01, 0.005
    for uh0 in (spectral.dft3(workloads.taylor_green(N)), ic.random_isotropic(N, seed=1001)):
        E_ref = []
        orc = spectral.Solver(N, nu, dt, integrator="euler").set_spectral(uh0).step(
            10, callback=lambda o: E_ref.append(o.energy()))
        s = _solver(N, nu, dt, integrator="euler", diag_every=1).set_spectral(to_dev(uh0, "f64")).step(10)
        assert spectral_rel_l2(to_host(s.get_spectral()), orc.uh) <= TOL_STEP10
        E, _ = s.history()
        assert np.max(np.abs(np.array(E) - E_ref) / np.array(E_ref)) <= 1e-12
        s.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_forward_euler_fused_matches_unfused_and_fp32(dtype):
    """The fused Euler step (RHS pass + next step's inverse x pass) gives the
    unfused schedule's bits; FP32 energy within 1e-5 of the oracle."""
    note(f"euler fused vs unfused {dtype}")
    N, nu, dt = 32, 0.01, 0.005
    uh0 = ic.random_isotropic(N, seed=1002)
    a = _solver(N, nu, dt, dtype=dtype, integrator="euler", fuse=True).set_spectral(to_dev(uh0, dtype)).step(4)
    b = _solver(N, nu, dt, dtype=dtype, integrator="euler", fuse=False).set_spectral(to_dev(uh0, dtype)).step(4)
    assert np.array_equal(to_host(a.get_spectral()), to_host(b.get_spectral()))
    if dtype == "f32":
        orc = spectral.Solver(N, nu, dt, integrator="euler").set_spectral(
            uh0.astype(np.complex64).astype(np.complex128)).step(4)
        assert abs(a.energy() - orc.energy()) / orc.energy() <= 1e-5


def test_autotuned_plan_is_cached():
    """dns_autotune stores its plan; a context created with autotune reuses
    the cached plan for the same (N, dtype) and gives the same bits."""
    import paper_1602_03638_amd as dns
    note("plan cache")
    dns.plan_cache_clear()
    N = 32
    uh0 = ic.random_isotropic(N, seed=1006)
    a = _solver(N, autotune=True)
    assert dns.plan_cache_entries() == 1
    b = _solver(N, autotune=True)
    assert dns.plan_cache_entries() == 1
    assert a.plan() == b.plan()
    c = _solver(N, dtype="f32", autotune=True)
    assert dns.plan_cache_entries() == 2
    a.set_spectral(to_dev(uh0, "f64")).step(2)
    b.set_spectral(to_dev(uh0, "f64")).step(2)
    assert np.array_equal(to_host(a.get_spectral()), to_host(b.get_spectral()))
    for s in (a, b, c):
        s.close()
    dns.plan_cache_clear()
    assert dns.plan_cache_entries() == 0


def test_plan_cache_persists_across_processes(tmp_path):
    """A tuned plan saved to a file and read back is taken by a new context
    (same variants, same bits); with DNS_PLAN_CACHE set, one process's
    autotune is written to the file and a second process reuses it."""
    import os
    import subprocess
    import sys
    import paper_1602_03638_amd as dns
    note("plan cache file")
    dns.plan_cache_clear()
    N = 64
    a = _solver(N, dtype="f32", autotune=True)
    plan = a.schedule()
    path = str(tmp_path / "plans.json")
    dns.plan_cache_save(path)
    dns.plan_cache_clear()
    assert dns.plan_cache_load(path) == 1
    b = _solver(N, dtype="f32", autotune=True)
    assert b.schedule() == plan and dns.plan_cache_entries() == 1
    uh0 = ic.random_isotropic(N, seed=1009)
    ra = to_host(a.set_spectral(to_dev(uh0, "f32")).step(2).get_spectral())
    rb = to_host(b.set_spectral(to_dev(uh0, "f32")).step(2).get_spectral())
    assert np.array_equal(ra, rb)
    a.close()
    b.close()
    f = _solver(N, dtype="f32", autotune="fastest")      # a cache entry of its own
    fast = f.schedule()
    assert dns.plan_cache_entries() == 2
    f.close()
    dns.plan_cache_save(path)
    dns.plan_cache_clear()
    assert dns.plan_cache_load(path) == 2
    g = _solver(N, dtype="f32", autotune="fastest")
    assert g.schedule() == fast and dns.plan_cache_entries() == 2
    g.close()
    dns.plan_cache_clear()
    env_path = str(tmp_path / "env_plans.json")
    child = ("import json, sys; sys.path.insert(0, %r); import paper_1602_03638_amd as d; "
             "s = d.Solver(32, 0.01, 0.005, autotune=True); n = d.plan_cache_entries(); "
             "print(json.dumps([n, s.schedule()]))") % (os.path.dirname(os.path.dirname(os.path.abspath(__file__))),)
    env = dict(os.environ, DNS_PLAN_CACHE=env_path)
    first = subprocess.run([sys.executable, "-c", child], env=env, capture_output=True, text=True, timeout=120)
    assert first.returncode == 0, first.stderr[-2000:]
    assert os.path.exists(env_path)
    second = subprocess.run([sys.executable, "-c", child], env=env, capture_output=True, text=True, timeout=120)
    assert second.returncode == 0, second.stderr[-2000:]
    n1, s1 = json.loads(first.stdout.strip().splitlines()[-1])
    n2, s2 = json.loads(second.stdout.strip().splitlines()[-1])
    assert n1 == 1 and n2 == 1 and s1 == s2


def test_caller_workspace_matches_library_allocation():
    """A context in a workspace from torch's allocator computes the same bits
    as one whose memory the library allocates; undersized or misaligned
    workspaces are rejected."""
    import torch
    import paper_1602_03638_amd as dns
    from paper_1602_03638_amd import DnsError
    note("caller workspace")
    N, nu, dt = 32, 0.01, 0.005
    uh0 = ic.random_isotropic(N, seed=1007)
    a = _solver(N, nu, dt, diag_every=1, workspace="torch").set_spectral(to_dev(uh0, "f64")).step(3)
    b = _solver(N, nu, dt, diag_every=1).set_spectral(to_dev(uh0, "f64")).step(3)
    assert np.array_equal(to_host(a.get_spectral()), to_host(b.get_spectral()))
    assert a.history() == b.history()
    a.close()
    b.close()
    need = dns.workspace_bytes(N, dns.DNS_FP64)
    small = torch.empty(need - 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(DnsError) as e:
        _solver(N, workspace=small)
    assert e.value.status == dns.DNS_E_INVAL
    big = torch.empty(need + 1024, dtype=torch.uint8, device="cuda")
    with pytest.raises(DnsError) as e:
        _solver(N, workspace=big[1:])                 # not 256-byte aligned
    assert e.value.status == dns.DNS_E_INVAL


def test_injected_launch_failure_reports_hip_error(monkeypatch):
    """DNS_FAULT_INJECT=launch makes the context's launch checks report
    DNS_E_HIP with a message; a context created without it is unaffected."""
    from paper_1602_03638_amd import DNS_E_HIP, DnsError
    note("fault injection")
    uh0 = ic.random_isotropic(16, seed=1008)
    monkeypatch.setenv("DNS_FAULT_INJECT", "launch")
    s = _solver(16)
    monkeypatch.delenv("DNS_FAULT_INJECT")
    with pytest.raises(DnsError) as e:
        s.set_spectral(to_dev(uh0, "f64"))
    assert e.value.status == DNS_E_HIP and "injected" in str(e.value)
    s.close()
    ok = _solver(16).set_spectral(to_dev(uh0, "f64")).step(1)
    assert np.isfinite(ok.energy())


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_nyquist_planes_of_masked_fields_stay_zero(dtype):
    """A field inside the 2/3-rule mask keeps its kz = N/2 plane (and the
    kx = -N/2, ky = -N/2 planes) exactly zero through RK4 steps: the mask
    removes the nonlinear term there and the viscous term of a zero mode is
    zero.  So the paper's pencil-solver choice of not storing the kz = N/2
    plane (Sec. 3.3) would leave these runs bit for bit unchanged."""
    note(f"nyquist planes stay zero {dtype}")
    N = 64
    s = _solver(N, 0.01, 0.005, dtype=dtype).init_random(1234, k0=4.0, energy=0.5).step(10)
    uh = to_host(s.get_spectral())
    assert np.count_nonzero(uh[:, :, :, N // 2]) == 0
    assert np.count_nonzero(uh[:, N // 2, :, :]) == 0 and np.count_nonzero(uh[:, :, N // 2, :]) == 0
    assert np.count_nonzero(uh) > 0
    s.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_variant_tables(dtype):
    """The plan dimensions each size offers: radix plan 1 (remainder stage
    first) exactly where log2 N is not a multiple of 3, plan 2 (radix-4
    stages) where it differs from plans 0 and 1 (not at 8 and 32), each on
    every pass; the z pass with no pad and pads 4, 8 and 16 at its default
    width; defaults on plan 0 with the z pad 8; every descriptor's radix and
    pad in range."""
    note(f"variant tables {dtype}")
    for N in (8, 16, 32, 64, 128, 256):
        s = _solver(N, dtype=dtype)
        var, sched = s.plan_variants_ex(), s.schedule()
        l = N.bit_length() - 1
        want = {1: l % 3 != 0, 2: N not in (8, 32)}
        for rs, present in want.items():
            for p, vs in var.items():
                assert any(d["radix"] == rs for d in vs) == present, (N, p, rs)
        zw = sched["zcross"]["width"]
        pads = {d["lds_pad"] for d in var["zcross"] if d["width"] == zw and d["radix"] == 0}
        assert pads == {0, 4, 8, 16}, (N, pads)
        assert all(d["radix"] == 0 for d in sched.values()) and sched["zcross"]["lds_pad"] == 8
        for p, vs in var.items():
            assert all(d["radix"] in (0, 1, 2) for d in vs)
            assert all(d["lds_pad"] == 0 for d in vs) or p == "zcross"
        s.close()
