"""Closed-form and seeded random input fields (see the package docstring)."""
import numpy as np


def mesh_1d(N):
    """x_i = 2 pi i / N, i = 0..N-1 (Sec. 2, eq. realmesh)."""
    return 2.0 * np.pi * np.arange(N, dtype=np.float64) / N


def _grid(N):
    x = mesh_1d(N)
    return x[:, None, None], x[None, :, None], x[None, None, :]


def taylor_green(N, dtype=np.float64):
    """Taylor-Green vortex u = sin x cos y cos z, v = -cos x sin y cos z, w = 0
    (Sec. 4.2 initial condition and the Appendix solver)."""
    X, Y, Z = _grid(N)
    u = np.empty((3, N, N, N), dtype=np.float64)
    u[0] = np.sin(X) * np.cos(Y) * np.cos(Z)
    u[1] = -np.cos(X) * np.sin(Y) * np.cos(Z)
    u[2] = 0.0
    return u.astype(dtype, copy=False)


def taylor_green_2d(N):
    """Planar Taylor-Green cell u = sin x cos y, v = -cos x sin y, w = 0."""
    X, Y, Z = _grid(N)
    u = np.zeros((3, N, N, N), dtype=np.float64)
    u[0] = np.sin(X) * np.cos(Y) + 0.0 * Z
    u[1] = -np.cos(X) * np.sin(Y) + 0.0 * Z
    return u


def abc_flow(N, A=1.0, B=1.0, C=1.0):
    """Arnold-Beltrami-Childress flow
    u = (A sin z + C cos y, B sin x + A cos z, C sin y + B cos x)."""
    X, Y, Z = _grid(N)
    u = np.empty((3, N, N, N), dtype=np.float64)
    u[0] = A * np.sin(Z) + C * np.cos(Y) + 0.0 * X
    u[1] = B * np.sin(X) + A * np.cos(Z) + 0.0 * Y
    u[2] = C * np.sin(Y) + B * np.cos(X) + 0.0 * Z
    return u


def shear_mode(N, k=1, amp=1.0):
    """Single shear wave u = (amp sin(k z), 0, 0)."""
    X, Y, Z = _grid(N)
    u = np.zeros((3, N, N, N), dtype=np.float64)
    u[0] = amp * np.sin(k * Z) + 0.0 * X + 0.0 * Y
    return u


def random_physical(N, seed, ncomp=3):
    """Seeded standard-normal real field (ncomp, N, N, N) float64."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((ncomp, N, N, N))


def random_half_spectrum(N, seed, ncomp=3):
    """Seeded complex array (ncomp, N, N, N/2+1) with standard-normal real and
    imaginary parts; not Hermitian on the kz = 0 and kz = N/2 planes."""
    rng = np.random.default_rng(seed)
    shape = (ncomp, N, N, N // 2 + 1)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


# The workloads the measurements and parity tests use (sizes, viscosity,
# time step, step count, precision).
CONFIGS = {
    "tg32_fp64": dict(ic="taylor_green", N=32, nu=0.01, dt=0.01, steps=10, dtype="f64"),
    "tg256_fp64": dict(ic="taylor_green", N=256, nu=1.0 / 1600, dt=1e-3, steps=100, dtype="f64"),
    "tg512": dict(ic="taylor_green", N=512, nu=1.0 / 1600, dt=1e-3, steps=50, dtype=("f64", "f32")),
    "iso1024_fp32": dict(ic="random_isotropic", N=1024, nu=1e-3, dt=5e-4, steps=20, dtype="f32", seed=1),
    "ensemble_fp32": dict(ic="random_isotropic", members=((32, 64), (64, 16), (128, 4)),
                          nu=0.01, dt=0.005, steps=100, dtype="f32", seed0=1000),
    "appendix_tg128": dict(ic="taylor_green", N=128, nu=0.000625, dt=0.01, steps=10, dtype="f64"),
}
