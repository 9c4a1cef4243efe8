"""Plain FP64 statement of the paper's spectral Navier-Stokes RK4 step.

TEST INFRASTRUCTURE ONLY (see the package docstring): imported by tests, the
smoke check and the CPU-baseline leg of the benchmark, never by the GPU path.

Notation follows Mortensen & Langtangen, arXiv:1602.03638:
  * physical mesh x_i = 2*pi*i/N, i = 0..N-1 on each axis (Sec. 2, eq. realmesh);
  * spectral storage order (Sec. 3.1, wavenumber-mesh listing):
    kx = ky = (0..N/2-1, -N/2..-1), kz = (0..N/2) with the last entry +N/2;
  * forward transform u_hat = sum_x u exp(-i k.x), unnormalised; inverse
    u = N^-3 sum_k u_hat exp(+i k.x) (Sec. 2, eqs. ffteq/iffteq), computed
    axis by axis: forward z (real) then y then x, inverse in reverse order
    (Sec. 2, eqs. fft/ifft);
  * the inverse real transform along z ignores the imaginary parts of the
    kz = 0 and kz = N/2 coefficients (the semantics of numpy's irfftn, which
    the paper's serial solver calls in Sec. 3.1).

Arrays: physical fields (3, N, N, N) float64 indexed [c, i, j, k] = (x, y, z);
spectral fields (3, N, N, N/2+1) complex128 indexed [c, ix, iy, iz].
"""
import numpy as np

_TWO_PI = 2.0 * np.pi


# ----------------------------------------------------------------------------
# Wavenumbers (Sec. 2: k in the set of eq. kmesh; Sec. 3.1: storage order)
# ----------------------------------------------------------------------------
def wavenumbers(N):
    """Integer wavenumber vectors (kx, ky, kz) in storage order (Sec. 3.1).

    kx = ky follow numpy's fftfreq(N, 1/N); kz is the first N/2+1 of those
    with the sign of the last one flipped, i.e. kz[N/2] = +N/2.
    """
    if N < 2 or N % 2:
        raise ValueError("N must be even")
    kx = np.concatenate([np.arange(0, N // 2), np.arange(-(N // 2), 0)]).astype(np.int64)
    kz = np.arange(0, N // 2 + 1, dtype=np.int64)
    return kx, kx.copy(), kz


def wavenumber_mesh(N):
    """The wavenumber vector of every stored mode and its squared length.

    Returns (K, K2): K[c, ix, iy, iz] is component c of k at storage index
    (ix, iy, iz), int64 of shape (3, N, N, N/2+1); K2 = |k|^2, int64 of shape
    (N, N, N/2+1), exact.
    """
    kx, ky, kz = wavenumbers(N)
    shape = (N, N, N // 2 + 1)
    K = np.stack([np.broadcast_to(kx[:, None, None], shape), np.broadcast_to(ky[None, :, None], shape),
                  np.broadcast_to(kz[None, None, :], shape)]).astype(np.int64)
    K2 = kx[:, None, None] ** 2 + ky[None, :, None] ** 2 + kz[None, None, :] ** 2
    return K, K2.astype(np.int64)


def dealias_mask(N, rule="text"):
    """2/3-rule cube mask (Sec. 3.1 dealias listing), shape (N, N, N/2+1) bool.

    A mode is kept iff |k_i| < kmax on all three axes.  rule="text" uses
    kmax = N/3 (the listing next to the 2/3-rule description); rule="appendix"
    uses kmax = 2/3 (N/2 + 1) (the Appendix solver).  Both comparisons are done
    exactly in integers: 3|k| < N, resp. 3|k| < N + 2.
    """
    kx, ky, kz = wavenumbers(N)
    if rule == "text":
        lim = N
    elif rule == "appendix":
        lim = N + 2
    else:
        raise ValueError("rule must be 'text' or 'appendix'")
    keep_x = 3 * np.abs(kx) < lim
    keep_y = 3 * np.abs(ky) < lim
    keep_z = 3 * np.abs(kz) < lim
    return keep_x[:, None, None] & keep_y[None, :, None] & keep_z[None, None, :]


# ----------------------------------------------------------------------------
# Discrete Fourier transforms by definition (Sec. 2, eqs. ffteq/iffteq/fft/ifft)
# ----------------------------------------------------------------------------
def _unit_root_table(N):
    """exp(-2 pi i r / N) for r = 0..N-1, exact at the quarter points."""
    r = np.arange(N)
    ang = _TWO_PI * r / N
    c = np.cos(ang)
    s = -np.sin(ang)
    # exp(-2 pi i r/N) is exactly 1, -i, -1, +i at r = 0, N/4, N/2, 3N/4
    if N % 4 == 0:
        q = N // 4
        c[0], s[0] = 1.0, 0.0
        c[q], s[q] = 0.0, -1.0
        c[2 * q], s[2 * q] = -1.0, 0.0
        c[3 * q], s[3 * q] = 0.0, 1.0
    elif N % 2 == 0:
        c[0], s[0] = 1.0, 0.0
        c[N // 2], s[N // 2] = -1.0, 0.0
    return c + 1j * s


def dft_matrix(N):
    """F[m, n] = exp(-2 pi i ((m n) mod N) / N): the forward DFT matrix.

    The product m*n is reduced modulo N in integers before any angle is
    formed, so every entry is one of the N exact N-th roots of unity.
    """
    m = np.arange(N, dtype=np.int64)
    r = np.outer(m, m) % N
    return _unit_root_table(N)[r]


def _c2r_matrices(N):
    """Real matrices (Cz, Sz), shape (N/2+1, N), for the inverse real DFT.

    u[n] = (1/N) [Re a_0 + (-1)^n Re a_{N/2}
                  + 2 sum_{m=1}^{N/2-1} Re(a_m exp(2 pi i m n / N))]
         = sum_m Re(a_m) Cz[m, n] + Im(a_m) Sz[m, n].
    Rows 0 and N/2 of Sz are zero: the imaginary parts of those two
    coefficients do not enter (numpy irfft semantics).
    """
    F = dft_matrix(N)[: N // 2 + 1, :]   # exp(-i ...): its conjugate is exp(+i ...)
    w = np.full(N // 2 + 1, 2.0)
    w[0] = 1.0
    w[N // 2] = 1.0
    Cz = (w[:, None] * F.real) / N           # Re(a e^{+i t}) = Re a cos t - Im a sin t
    Sz = (w[:, None] * F.imag) / N           # F.imag = -sin t
    Sz[0, :] = 0.0
    Sz[N // 2, :] = 0.0
    return Cz, Sz


def _apply_x(M, a):
    """Contract matrix M (P, N) with axis -3 of a (..., N, N2, N3)."""
    lead = a.shape[:-3]
    n, n2, n3 = a.shape[-3:]
    flat = np.ascontiguousarray(a).reshape((-1, n, n2 * n3))
    out = np.matmul(M, flat)
    return out.reshape(lead + (M.shape[0], n2, n3))


def _apply_y(M, a):
    """Contract matrix M (P, N) with axis -2 of a (..., N1, N, N3)."""
    return np.matmul(M, np.ascontiguousarray(a))


def _apply_z(M, a):
    """Contract matrix M (P, N) with the last axis of a (..., N)."""
    lead = a.shape[:-1]
    flat = np.ascontiguousarray(a).reshape((-1, a.shape[-1]))
    return (flat @ M.T).reshape(lead + (M.shape[0],))


def dft3(u):
    """Forward real 3D DFT over the last three axes (Sec. 2, eq. fft).

    u: real array (..., N, N, N).  Returns complex (..., N, N, N/2+1):
    uh[kx, ky, kz] = sum_{x,y,z} u[x,y,z] exp(-i (kx x + ky y + kz z)),
    computed as the real transform along z, then the complex one along y,
    then along x.  Unnormalised.
    """
    u = np.asarray(u, dtype=np.float64)
    N = u.shape[-1]
    if u.shape[-3:] != (N, N, N):
        raise ValueError("expected (..., N, N, N)")
    F = dft_matrix(N)
    Fr = F[: N // 2 + 1, :]
    a = _apply_z(Fr, u)               # z: (..., x, y, kz)
    a = _apply_y(F, a)                # y: (..., x, ky, kz)
    a = _apply_x(F, a)                # x: (..., kx, ky, kz)
    return a


def idft3(uh):
    """Inverse real 3D DFT over the last three axes (Sec. 2, eq. ifft).

    uh: complex (..., N, N, N/2+1).  Returns real (..., N, N, N):
    complex inverse along x, then along y (each with 1/N), then the inverse
    real transform along z (with 1/N), which ignores Im of kz = 0 and N/2.
    """
    uh = np.asarray(uh, dtype=np.complex128)
    N = uh.shape[-3]
    if uh.shape[-3:] != (N, N, N // 2 + 1):
        raise ValueError("expected (..., N, N, N/2+1)")
    Finv = np.conj(dft_matrix(N)) / N
    a = _apply_x(Finv, uh)            # x
    a = _apply_y(Finv, a)             # y
    Cz, Sz = _c2r_matrices(N)
    return _apply_z(Cz.T, np.ascontiguousarray(a.real)) + _apply_z(Sz.T, np.ascontiguousarray(a.imag))  # z (c2r)


def idft3_point(uh, i, j, l):
    """u at the mesh point (x_i, y_j, z_l) of the inverse transform idft3(uh),
    evaluated by the definition for that one point (spot checks of inverse
    transforms too large to evaluate whole):
      a(kz) = N^-2 sum_{kx, ky} u_hat[kx, ky, kz] exp(+i (kx x_i + ky y_j)),
      u = N^-1 [Re a(0) + (-1)^l Re a(N/2) + 2 sum_{0 < kz < N/2} Re(a(kz) exp(+i kz z_l))],
    which keeps numpy irfftn's treatment of the kz = 0 and N/2 coefficients
    (their imaginary parts after the x and y sums do not enter).  Angles are
    reduced modulo N in integers.  uh: (..., N, N, N/2+1)."""
    uh = np.asarray(uh, dtype=np.complex128)
    N = uh.shape[-3]
    roots = np.conj(_unit_root_table(N))            # exp(+2 pi i r / N)
    n = np.arange(N, dtype=np.int64)
    ex = roots[(n * i) % N]                          # over storage index ix (kx = ix mod N)
    ey = roots[(n * j) % N]
    a = np.tensordot(np.tensordot(uh, ex, axes=([-3], [0])), ey, axes=([-2], [0])) / float(N) ** 2
    M = N // 2
    ez = roots[(np.arange(M + 1, dtype=np.int64) * l) % N]
    t = np.real(a * ez)
    w = np.full(M + 1, 2.0)
    w[0] = 1.0
    w[M] = 1.0
    t[..., 0] = np.real(a[..., 0])
    t[..., M] = np.real(a[..., M]) * (1.0 if l % 2 == 0 else -1.0)
    return np.sum(w * t, axis=-1) / N


def dft3_mode(u, ix, iy, iz):
    """One coefficient of dft3(u) by the definition, for spot checks of
    transforms too large to evaluate whole: u_hat[ix, iy, iz] =
    sum_{x,y,z} u[x,y,z] exp(-2 pi i ((ix x + iy y + iz z) mod N) / N),
    summed over z, then y, then x with exact reduced twiddles."""
    u = np.asarray(u, dtype=np.float64)
    N = u.shape[-1]
    roots = _unit_root_table(N)
    n = np.arange(N, dtype=np.int64)
    ez = roots[(iz * n) % N]
    ey = roots[(iy * n) % N]
    ex = roots[(ix * n) % N]
    a = u @ ez           # (..., N, N)
    b = a @ ey           # (..., N)
    return b @ ex


# ----------------------------------------------------------------------------
# The right-hand side (Sec. 2 eqs. NSf, mod_pressure, NSfinal, curl_convection;
# Sec. 3.1 Curl, Cross and computeRHS listings)
# ----------------------------------------------------------------------------
def curl_hat(uh, K):
    """omega_hat = i k x u_hat (Sec. 3.1, curl equation and Curl listing)."""
    w = np.empty_like(uh)
    w[0] = 1j * (K[1] * uh[2] - K[2] * uh[1])
    w[1] = 1j * (K[2] * uh[0] - K[0] * uh[2])
    w[2] = 1j * (K[0] * uh[1] - K[1] * uh[0])
    return w


def cross(a, b):
    """c = a x b, componentwise on the leading axis (Sec. 3.4 cross listing)."""
    c = np.empty_like(a)
    c[0] = a[1] * b[2] - a[2] * b[1]
    c[1] = a[2] * b[0] - a[0] * b[2]
    c[2] = a[0] * b[1] - a[1] * b[0]
    return c


def project(n, K, K2):
    """Divergence-free part of n at every mode (eqs. mod_pressure, NSfinal):
    the pressure gradient removes the component along k,
      P(n) = n - k (k . n) / |k|^2,
    and leaves the k = 0 mode unchanged (it has no pressure)."""
    kn = K[0] * n[0] + K[1] * n[1] + K[2] * n[2]
    along = np.where(K2 > 0, kn / np.where(K2 > 0, K2, 1), 0.0)
    return n - K * along


def nonlinear_hat(uh, K, mask):
    """The dealiased convection term of eq. NSfinal: F(u x omega) with
    u = F^-1(u_hat), omega = F^-1(i k x u_hat) (eq. curl_convection), set to
    zero outside the 2/3-rule mask (Sec. 3.1)."""
    u = idft3(uh)
    omega = idft3(curl_hat(uh, K))
    return mask * dft3(cross(u, omega))


def rhs(uh, nu, mesh, mask):
    """d u_hat / dt of eq. NSfinal: the projected dealiased convection term
    minus the viscous term nu |k|^2 u_hat.  The velocity is obtained from
    u_hat at every evaluation."""
    K, K2 = mesh
    return project(nonlinear_hat(uh, K, mask), K, K2) - nu * K2 * uh


def rk4_step(uh, nu, dt, mesh, mask):
    """One step of the classical fourth-order Runge-Kutta method, the
    integrator of the Appendix solver:
      k1 = f(u), k2 = f(u + dt/2 k1), k3 = f(u + dt/2 k2), k4 = f(u + dt k3),
      u_new = u + dt/6 (k1 + 2 k2 + 2 k3 + k4),  f = rhs."""
    def f(v):
        return rhs(v, nu, mesh, mask)
    k1 = f(uh)
    k2 = f(uh + (dt / 2) * k1)
    k3 = f(uh + (dt / 2) * k2)
    k4 = f(uh + dt * k3)
    return uh + (dt / 6) * (k1 + 2 * k2 + 2 * k3 + k4)


def euler_step(uh, nu, dt, mesh, mask):
    """One forward Euler step, the time loop of the Sec. 3.1 listing:
    u_new = u + dt f(u), f = rhs."""
    return uh + dt * rhs(uh, nu, mesh, mask)


# ----------------------------------------------------------------------------
# Diagnostics (Appendix: energy reduce; Sec. 4.2: energy and vorticity)
# ----------------------------------------------------------------------------
def _hermitian_weight(N):
    """Weight of each stored kz column in a full-spectrum sum: 1 at kz = 0
    and kz = N/2 (their mirrors are themselves), 2 elsewhere."""
    w = np.full(N // 2 + 1, 2.0)
    w[0] = 1.0
    w[N // 2] = 1.0
    return w


def energy(uh):
    """E = mean over the mesh of |u|^2 / 2, from the half spectrum (Parseval):
    E = (1 / 2N^6) sum_k w |u_hat|^2 over all three components."""
    N = uh.shape[-3]
    w = _hermitian_weight(N)
    return float(np.sum(w * np.abs(uh) ** 2) / (2.0 * float(N) ** 6))


def enstrophy(uh):
    """Omega = mean over the mesh of |omega|^2 / 2 = (1/2N^6) sum_k w |k x u_hat|^2."""
    N = uh.shape[-3]
    K, _ = wavenumber_mesh(N)
    return energy(curl_hat(uh, K))


def energy_physical(u):
    """E = 0.5 * sum(u*u) / N^3, the Appendix's final energy reduction."""
    N = u.shape[-1]
    return float(0.5 * np.sum(u * u) / float(N) ** 3)


def divergence_max(uh):
    """Relative size of the divergence, max_k |k . u_hat(k)| / (max |k| *
    max |u_hat|), over the stored modes: 0 for a solenoidal field (the
    spectral form of div u = 0, Sec. 2)."""
    N = uh.shape[-3]
    K, K2 = wavenumber_mesh(N)
    div = np.abs(K[0] * uh[0] + K[1] * uh[1] + K[2] * uh[2])
    scale = np.sqrt(float(np.max(K2))) * np.max(np.abs(uh))
    return float(np.max(div) / scale) if scale > 0 else 0.0


class Solver:
    """Holds u_hat and advances it with rk4_step (or euler_step); mirrors the
    C ABI calls.

    Solver(N, nu, dt, rule, integrator).set_velocity(u) / set_spectral(uh);
    step(n); energy(); enstrophy(); get_velocity(); get_spectral().
    integrator: "rk4" (Appendix solver, default) or "euler" (Sec. 3.1 loop).
    """

    def __init__(self, N, nu, dt, rule="text", integrator="rk4"):
        self.N, self.nu, self.dt = int(N), float(nu), float(dt)
        self._step = {"rk4": rk4_step, "euler": euler_step}[integrator]
        self.mesh = wavenumber_mesh(self.N)
        self.mask = dealias_mask(self.N, rule)
        self.uh = None
        self.steps = 0

    def set_velocity(self, u):
        self.uh = dft3(u)
        return self

    def set_spectral(self, uh):
        self.uh = np.array(uh, dtype=np.complex128)
        return self

    def step(self, n=1, callback=None):
        for _ in range(int(n)):
            self.uh = self._step(self.uh, self.nu, self.dt, self.mesh, self.mask)
            self.steps += 1
            if callback is not None:
                callback(self)
        return self

    def get_spectral(self):
        return self.uh.copy()

    def get_velocity(self):
        return idft3(self.uh)

    def energy(self):
        return energy(self.uh)

    def enstrophy(self):
        return enstrophy(self.uh)
