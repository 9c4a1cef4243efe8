"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each pin returns an error measure; tests/test_oracle_pins.py asserts each one
is within its tolerance and tests/test_oracle_mutations.py plants plausible
mistakes in the oracle and asserts that some pin then fails.  Nothing here
re-types the oracle's own formulas: each pin compares against brute force, a
closed form, an invariant or a value printed in the paper.
"""
import json
import os

import numpy as np

import workloads
from oracle import ic, spectral

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

TOL = {
    "dealias_table": 0.0,
    "mesh_listing": 0.0,
    "brute_dft": 1e-14,
    "brute_idft": 1e-14,
    "numpy_fft": 1e-14,
    "parseval": 1e-14,
    "roundtrip": 1e-14,
    "abc_curl": 1e-14,
    "abc_rhs": 1e-14,
    "tg2d_rhs": 1e-14,
    "tg_initial_tendency": 1e-14,
    "tg_initial_diagnostics": 1e-15,
    "rk4_decay": 1e-14,
    "euler_decay": 1e-14,
    "masked_linear": 1e-14,
    "divergence": 1e-13,
    "divergence_closed_form": 1e-14,
    "point_inverse": 1e-14,
    "energy_budget": 1e-7,
    "appendix": 5e-13,
    "rk4_order_lo": 14.0,
    "rk4_order_hi": 18.0,
    "euler_order_lo": 1.8,
    "euler_order_hi": 2.2,
}


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


# ---------------------------------------------------------------- transforms
def brute_dft_error(N=8, seed=11):
    """Triple-sum 3D DFT of an asymmetric random field, by direct summation
    over all N^3 points for every stored mode (eq. iffteq)."""
    u = workloads.random_physical(N, seed, ncomp=1)[0]
    x = np.arange(N)
    kx, ky, kz = spectral.wavenumbers(N)
    ref = np.zeros((N, N, N // 2 + 1), dtype=np.complex128)
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    for a in range(N):
        for b in range(N):
            for c in range(N // 2 + 1):
                phase = 2.0 * np.pi * (kx[a] * X + ky[b] * Y + kz[c] * Z) / N
                ref[a, b, c] = np.sum(u * np.exp(-1j * phase))
    return _rel(spectral.dft3(u), ref)


def brute_idft_error(N=8, seed=12):
    """Inverse by direct summation over the full spectrum (eq. ffteq): the
    half spectrum of a real field is extended by Hermitian symmetry."""
    u = workloads.random_physical(N, seed, ncomp=1)[0]
    uh = spectral.dft3(u)
    full = np.zeros((N, N, N), dtype=np.complex128)
    full[:, :, : N // 2 + 1] = uh
    for c in range(N // 2 + 1, N):
        full[:, :, c] = np.conj(uh[(-np.arange(N)) % N][:, (-np.arange(N)) % N, N - c])
    x = np.arange(N)
    k = np.concatenate([np.arange(0, N // 2), np.arange(-(N // 2), 0)])
    ref = np.zeros((N, N, N))
    KX, KY, KZ = np.meshgrid(k, k, k, indexing="ij")
    for i in range(N):
        for j in range(N):
            for l in range(N):
                phase = 2.0 * np.pi * (KX * x[i] + KY * x[j] + KZ * x[l]) / N
                ref[i, j, l] = np.real(np.sum(full * np.exp(1j * phase))) / N ** 3
    return _rel(spectral.idft3(uh), ref)


def numpy_fft_error(N=32, seed=13):
    """numpy.fft.rfftn / irfftn (the routines the paper's serial code calls)."""
    u = workloads.random_physical(N, seed)
    e1 = _rel(spectral.dft3(u), np.fft.rfftn(u, axes=(1, 2, 3)))
    h = workloads.random_half_spectrum(N, seed + 1)
    e2 = _rel(spectral.idft3(h), np.fft.irfftn(h, s=(N, N, N), axes=(1, 2, 3)))
    return max(e1, e2)


def parseval_error(N=16, seed=14):
    u = workloads.random_physical(N, seed)
    return abs(spectral.energy(spectral.dft3(u)) - spectral.energy_physical(u)) / spectral.energy_physical(u)


def roundtrip_error(N=16, seed=15):
    u = workloads.random_physical(N, seed)
    return _rel(spectral.idft3(spectral.dft3(u)), u)


# ---------------------------------------------------------------- meshes
def mesh_listing_error():
    """Wavenumber mesh against the storage order written out in Sec. 3.1
    (N = 8: kx = ky = 0,1,2,3,-4,-3,-2,-1 and kz = 0,1,2,3,+4)."""
    kxy = np.array([0, 1, 2, 3, -4, -3, -2, -1])
    kz = np.array([0, 1, 2, 3, 4])
    K, K2 = spectral.wavenumber_mesh(8)
    err = 0.0
    for a in range(8):
        for b in range(8):
            for c in range(5):
                k = np.array([kxy[a], kxy[b], kz[c]])
                k2 = int(k @ k)
                err = max(err, float(np.max(np.abs(K[:, a, b, c] - k))), abs(int(K2[a, b, c]) - k2))
    return err


def dealias_table_error():
    """Number of (rule, N) entries whose largest kept |k_i| differs from the
    hand-worked cutoff table (Sec. 3.1 listing, Appendix constant), or whose
    mask is not the cube product of its three 1D masks."""
    with open(os.path.join(GOLDEN, "dealias_cutoffs.json")) as f:
        table = json.load(f)["largest_kept"]
    bad = 0
    for rule, rows in table.items():
        for n_str, kmax in rows.items():
            N = int(n_str)
            mask = spectral.dealias_mask(N, rule)
            kx, _, kz = spectral.wavenumbers(N)
            keep_xy = np.abs(kx) <= kmax
            keep_z = np.abs(kz) <= kmax
            cube = keep_xy[:, None, None] & keep_xy[None, :, None] & keep_z[None, None, :]
            bad += int(not np.array_equal(mask, cube))
    return float(bad)


# ---------------------------------------------------------------- RHS pieces
def abc_curl_error(N=16):
    """The ABC flow is a Beltrami field: its vorticity equals the velocity."""
    u = workloads.abc_flow(N, 1.0, 0.7, 0.4)
    K, _ = spectral.wavenumber_mesh(N)
    w = spectral.idft3(spectral.curl_hat(spectral.dft3(u), K))
    return _rel(w, u)


def abc_rhs_error(N=16, nu=0.013):
    """u x omega = u x u = 0, and every mode has |k|^2 = 1: RHS = -nu u_hat."""
    uh = spectral.dft3(workloads.abc_flow(N, 1.0, 0.7, 0.4))
    r = spectral.rhs(uh, nu, spectral.wavenumber_mesh(N), spectral.dealias_mask(N))
    return float(np.max(np.abs(r + nu * uh)) / np.max(np.abs(uh)))


def tg2d_rhs_error(N=16, nu=0.021):
    """Planar Taylor-Green: u x omega is a pure gradient (removed by the
    pressure projection) and |k|^2 = 2: RHS = -2 nu u_hat."""
    uh = spectral.dft3(workloads.taylor_green_2d(N))
    r = spectral.rhs(uh, nu, spectral.wavenumber_mesh(N), spectral.dealias_mask(N))
    return float(np.max(np.abs(r + 2.0 * nu * uh)) / np.max(np.abs(uh)))


def tg_initial_tendency_error(N=16, nu=0.0173):
    """Closed-form time derivative of the 3D Taylor-Green field at t = 0.

    With u0 = (sin x cos y cos z, -cos x sin y cos z, 0), the initial
    pressure is p0 = (cos 2x + cos 2y)(cos 2z + 2)/16 and
    -u0.grad u0 - grad p0 = (-sin 2x cos 2z, -sin 2y cos 2z,
    (cos 2x + cos 2y) sin 2z) / 8, while nu lap u0 = -3 nu u0.  This pins
    the sign and layout of the curl, the cross product and the projection.
    """
    x = workloads.mesh_1d(N)
    X, Y, Z = x[:, None, None], x[None, :, None], x[None, None, :]
    D = np.empty((3, N, N, N))
    D[0] = -np.sin(2 * X) * np.cos(2 * Z) / 8 + 0 * Y
    D[1] = -np.sin(2 * Y) * np.cos(2 * Z) / 8 + 0 * X
    D[2] = (np.cos(2 * X) + np.cos(2 * Y)) * np.sin(2 * Z) / 8
    u0 = workloads.taylor_green(N)
    expect = spectral.dft3(D - 3.0 * nu * u0)
    r = spectral.rhs(spectral.dft3(u0), nu, spectral.wavenumber_mesh(N), spectral.dealias_mask(N))
    return float(np.max(np.abs(r - expect)) / np.max(np.abs(expect)))


def tg_initial_diagnostics_error(N=16):
    """E(0) = 1/8 and enstrophy(0) = 3/8 for the 3D Taylor-Green field."""
    uh = spectral.dft3(workloads.taylor_green(N))
    return max(abs(spectral.energy(uh) - 0.125) / 0.125,
               abs(spectral.enstrophy(uh) - 0.375) / 0.375)


def rk4_decay_error(N=16, nu=0.01, dt=0.01, steps=10):
    """Nonlinearity-free flows: every RK4 step multiplies the amplitude by
    R(z) = 1 + z + z^2/2 + z^3/6 + z^4/24 with z = -nu |k|^2 dt, so
    E_n / E_0 = R(z)^(2n) (|k|^2 = 1 for ABC, 2 for planar Taylor-Green)."""
    errs = []
    for field, k2 in ((workloads.abc_flow(N, 1.0, 0.7, 0.4), 1.0), (workloads.taylor_green_2d(N), 2.0)):
        s = spectral.Solver(N, nu, dt).set_velocity(field)
        e0 = s.energy()
        s.step(steps)
        z = -nu * k2 * dt
        R = 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24
        errs.append(abs(s.energy() / e0 - R ** (2 * steps)) / R ** (2 * steps))
    return max(errs)


def euler_decay_error(N=16, nu=0.01, dt=0.01, steps=10):
    """Forward Euler on nonlinearity-free flows multiplies the amplitude by
    1 + z per step, z = -nu |k|^2 dt, so E_n / E_0 = (1 + z)^(2n)."""
    errs = []
    for field, k2 in ((workloads.abc_flow(N, 1.0, 0.7, 0.4), 1.0), (workloads.taylor_green_2d(N), 2.0)):
        s = spectral.Solver(N, nu, dt, integrator="euler").set_velocity(field)
        e0 = s.energy()
        s.step(steps)
        g = (1 - nu * k2 * dt) ** (2 * steps)
        errs.append(abs(s.energy() / e0 - g) / g)
    return max(errs)


def euler_order_ratio(N=16, nu=0.05, T=0.05, seed=8):
    """Self-convergence of forward Euler: error(dt) / error(dt/2) ~ 2, against
    an RK4 run (whose error is negligible at this dt) on a nonlinear flow."""
    uh0 = ic.random_isotropic(N, seed, k0=3.0)
    ref = spectral.Solver(N, nu, T / 16).set_spectral(uh0).step(16).uh

    def run(n):
        return spectral.Solver(N, nu, T / n, integrator="euler").set_spectral(uh0).step(n).uh

    e1 = np.linalg.norm(run(8) - ref)
    e2 = np.linalg.norm(run(16) - ref)
    return float(e1 / e2)


def masked_linear_error(N=16, nu=0.02, seed=3):
    """Outside the dealias mask the nonlinear term is removed, so there
    RHS = -nu |k|^2 u_hat exactly; inside, RHS + nu |k|^2 u_hat is
    divergence-free (k . N_hat = 0 after the projection)."""
    uh = ic.random_isotropic(N, seed, k0=3.0)
    uh = uh + 0.05 * np.abs(uh).max() * spectral.dft3(workloads.random_physical(N, seed))
    mesh = spectral.wavenumber_mesh(N)
    K, K2 = mesh
    mask = spectral.dealias_mask(N)
    r = spectral.rhs(uh, nu, mesh, mask)
    nonlin = r + nu * K2 * uh
    scale = np.max(np.abs(nonlin))
    out = float(np.max(np.abs(nonlin[:, ~mask])) / scale)
    div = float(np.max(np.abs(np.sum(K * nonlin, axis=0))) / (scale * np.sqrt(K2.max())))
    return max(out, div)


# ---------------------------------------------------------------- solver
def divergence_error(N=16, nu=0.01, dt=0.01, steps=3, seed=5):
    s = spectral.Solver(N, nu, dt).set_spectral(ic.random_isotropic(N, seed, k0=3.0))
    s.step(steps)
    return spectral.divergence_max(s.uh)


def divergence_closed_form_error(N=16):
    """divergence_max of fields with a known divergence.  u = (sin x, 0, 0):
    u_hat_x = -+ i N^3/2 at kx = +-1, so max |k . u_hat| = N^3/2 = max |u_hat|,
    and the largest |k| on the stored mesh is sqrt(3) N/2 (kx = ky = -N/2,
    kz = +N/2): the value is 2 / (sqrt(3) N).  u = (0, 0, cos 2z): u_hat_z =
    N^3/2 at kz = 2 gives 4 / (sqrt(3) N).  u = (0, sin 3y, 0) + a solenoidal
    Taylor-Green field of larger amplitude: 6 / (sqrt(3) N) times N^3/2 over
    the largest coefficient.  A solenoidal field gives 0."""
    x = workloads.mesh_1d(N)
    X, Y, Z = x[:, None, None], x[None, :, None], x[None, None, :]
    zero = 0 * X + 0 * Y + 0 * Z
    errs = []
    u = np.stack([np.sin(X) + zero, zero, zero])
    errs.append(abs(spectral.divergence_max(spectral.dft3(u)) - 2 / (np.sqrt(3) * N)) / (2 / (np.sqrt(3) * N)))
    u = np.stack([zero, zero, np.cos(2 * Z) + zero])
    errs.append(abs(spectral.divergence_max(spectral.dft3(u)) - 4 / (np.sqrt(3) * N)) / (4 / (np.sqrt(3) * N)))
    tg = workloads.taylor_green(N)
    u = 4.0 * tg + np.stack([zero, np.sin(3 * Y) + zero, zero])
    uh = spectral.dft3(u)
    want = 3 * (N ** 3 / 2) / (np.sqrt(3) * N / 2 * np.max(np.abs(uh)))
    errs.append(abs(spectral.divergence_max(uh) - want) / want)
    errs.append(spectral.divergence_max(spectral.dft3(tg)))
    return max(errs)


def point_inverse_error(N=8, seed=21):
    """idft3_point at every mesh point against numpy.fft.irfftn (the routine
    the paper's serial code calls) of a random, not Hermitian, half
    spectrum, and against the closed form of a plane wave a cos(k . x + phi)
    whose transform is N^3 a e^{i phi} / 2 at k."""
    h = workloads.random_half_spectrum(N, seed)
    ref = np.fft.irfftn(h, s=(N, N, N), axes=(1, 2, 3))
    got = np.empty_like(ref)
    for i in range(N):
        for j in range(N):
            for l in range(N):
                got[:, i, j, l] = spectral.idft3_point(h, i, j, l)
    err = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
    M = 16
    kx, ky, kz, a, phi = 3, -5, 2, 0.75, 0.4
    wave = np.zeros((1, M, M, M // 2 + 1), dtype=np.complex128)
    wave[0, kx % M, ky % M, kz] = M ** 3 * a * np.exp(1j * phi) / 2
    for i, j, l in ((0, 0, 0), (1, 2, 3), (15, 7, 9), (4, 11, 15)):
        x = 2 * np.pi * np.array([i, j, l]) / M
        want = a * np.cos(kx * x[0] + ky * x[1] + kz * x[2] + phi)
        err = max(err, abs(float(spectral.idft3_point(wave, i, j, l)[0]) - want))
    return err


def energy_budget_error(N=32, nu=0.01, dt=0.01, steps=10):
    """Semi-discrete identity dE/dt = -2 nu Omega (u . (u x omega) = 0
    pointwise and Parseval is exact on the grid); trapezoid residual over
    the Taylor-Green run."""
    s = spectral.Solver(N, nu, dt).set_velocity(workloads.taylor_green(N))
    E = [s.energy()]
    W = [s.enstrophy()]
    for _ in range(steps):
        s.step(1)
        E.append(s.energy())
        W.append(s.enstrophy())
    res = [abs((E[n + 1] - E[n]) / dt + nu * (W[n] + W[n + 1])) for n in range(steps)]
    return max(res)


def rk4_order_ratio(N=16, nu=0.05, T=0.2, seed=8):
    """Self-convergence: error(dt) / error(dt/2) ~ 16 for a fourth-order
    method, measured against a dt/8 run on a random nonlinear flow."""
    uh0 = ic.random_isotropic(N, seed, k0=3.0)

    def run(n):
        return spectral.Solver(N, nu, T / n).set_spectral(uh0).step(n).uh

    ref = run(32)
    e1 = np.linalg.norm(run(4) - ref)
    e2 = np.linalg.norm(run(8) - ref)
    return float(e1 / e2)


def appendix_error():
    """The paper's worked example: final energy printed in the Appendix."""
    with open(os.path.join(GOLDEN, "appendix_tg128.json")) as f:
        g = json.load(f)
    N = g["N"]
    s = spectral.Solver(N, g["nu"], g["dt"], g["dealias"]).set_velocity(workloads.taylor_green(N))
    s.step(g["steps"])
    return abs(spectral.energy_physical(s.get_velocity()) - g["energy_printed"])


FAST_PINS = {
    "dealias_table": dealias_table_error,
    "mesh_listing": mesh_listing_error,
    "brute_dft": brute_dft_error,
    "brute_idft": brute_idft_error,
    "numpy_fft": numpy_fft_error,
    "parseval": parseval_error,
    "roundtrip": roundtrip_error,
    "abc_curl": abc_curl_error,
    "abc_rhs": abc_rhs_error,
    "tg2d_rhs": tg2d_rhs_error,
    "tg_initial_tendency": tg_initial_tendency_error,
    "tg_initial_diagnostics": tg_initial_diagnostics_error,
    "rk4_decay": rk4_decay_error,
    "euler_decay": euler_decay_error,
    "masked_linear": masked_linear_error,
    "divergence": divergence_error,
    "divergence_closed_form": divergence_closed_form_error,
    "point_inverse": point_inverse_error,
    "energy_budget": energy_budget_error,
}


def fast_pin_failures():
    """Names of the fast pins that fail (used by the planted-mistake test)."""
    bad = []
    for name, fn in FAST_PINS.items():
        try:
            err = fn()
        except Exception:  # a planted mistake may also break shapes
            bad.append(name)
            continue
        if not np.isfinite(err) or err > TOL[name]:
            bad.append(name)
    r = rk4_order_ratio()
    if not (TOL["rk4_order_lo"] <= r <= TOL["rk4_order_hi"]):
        bad.append("rk4_order")
    r = euler_order_ratio()
    if not (TOL["euler_order_lo"] <= r <= TOL["euler_order_hi"]):
        bad.append("euler_order")
    return bad
