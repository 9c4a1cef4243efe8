"""Plant plausible mistakes in the CPU oracle and check that the pins catch
each one: evidence that the pins constrain every part of the oracle
(transforms, curl, cross product, mask, projection, viscous term, RK4,
forward Euler, diagnostics).  Mistakes are planted on the CPU only, by monkeypatching."""
import numpy as np
import pytest

import oracle_pins as pins
from oracle import spectral

_orig = {name: getattr(spectral, name) for name in (
    "cross", "curl_hat", "rhs", "dft3", "idft3", "_unit_root_table", "project", "nonlinear_hat",
    "_c2r_matrices", "_hermitian_weight", "wavenumber_mesh", "dealias_mask", "divergence_max",
    "idft3_point")}


def _cross_swapped(a, b):
    return _orig["cross"](b, a)


def _curl_neg(uh, K):
    return -_orig["curl_hat"](uh, K)


def _curl_index_slip(uh, K):
    w = _orig["curl_hat"](uh, K)
    w[0] = 1j * (K[1] * uh[2] - K[2] * uh[0])
    return w


def _nonlinear_unmasked(uh, K, mask):
    return _orig["nonlinear_hat"](uh, K, np.ones_like(mask))


def _project_variant(kind):
    def project(n, K, K2):
        kn = K[0] * n[0] + K[1] * n[1] + K[2] * n[2]
        along = np.where(K2 > 0, kn / np.where(K2 > 0, K2, 1), 0.0)
        if kind == "none":
            return n.copy()
        if kind == "sign":
            return n + K * along
        return n - K[::-1] * along          # transposed
    return project


def _rhs_viscous(kind):
    def rhs(uh, nu, mesh, mask):
        K, K2 = mesh
        nl = spectral.project(spectral.nonlinear_hat(uh, K, mask), K, K2)
        return nl + nu * K2 * uh if kind == "sign" else nl - nu * np.sqrt(K2) * uh
    return rhs


def _roots_conj(N):
    return np.conj(_orig["_unit_root_table"](N))


def _c2r_no_weights(N):
    Cz, Sz = _orig["_c2r_matrices"](N)
    w = np.full(N // 2 + 1, 2.0)
    w[0] = w[-1] = 1.0
    return Cz / w[:, None], Sz / w[:, None]


def _idft_missing_norm(uh):
    return _orig["idft3"](uh) * uh.shape[-3]


def _dft_axes_swapped(u):
    return _orig["dft3"](np.swapaxes(u, -1, -3))


def _weights_flat(N):
    return np.full(N // 2 + 1, 2.0)


def _mesh_kz_nyquist_negative(N):
    K, K2 = _orig["wavenumber_mesh"](N)
    K = K.copy()
    K[2, :, :, -1] *= -1
    return K, K2


def _mask_round(N, rule="text"):
    kx, ky, kz = spectral.wavenumbers(N)
    lim = N / 3.0 + 1
    return (np.abs(kx)[:, None, None] < lim) & (np.abs(ky)[None, :, None] < lim) & (np.abs(kz)[None, None, :] < lim)


def _divergence_zero(uh):
    return 0.0


def _divergence_transposed(uh):
    N = uh.shape[-3]
    K, K2 = spectral.wavenumber_mesh(N)
    div = np.abs(K[2] * uh[0] + K[1] * uh[1] + K[0] * uh[2])
    return float(np.max(div) / (np.sqrt(float(np.max(K2))) * np.max(np.abs(uh))))


def _point_variant(uh, i, j, l):
    N = uh.shape[-3]
    h = np.array(uh, dtype=np.complex128, copy=True)
    if l % 2:
        h[..., N // 2] = -h[..., N // 2]      # undo the sign the helper applies to the kz = N/2 term
    return _orig["idft3_point"](h, i, j, l)


def _point_forward_sign(uh, i, j, l):
    N = uh.shape[-3]
    return _orig["idft3_point"](uh, (-i) % N, (-j) % N, (-l) % N)


MUTATIONS = {
    "cross_swapped": ("cross", _cross_swapped),
    "curl_negated": ("curl_hat", _curl_neg),
    "curl_index_slip": ("curl_hat", _curl_index_slip),
    "no_mask": ("nonlinear_hat", _nonlinear_unmasked),
    "no_projection": ("project", _project_variant("none")),
    "projection_sign": ("project", _project_variant("sign")),
    "projection_transposed": ("project", _project_variant("transposed")),
    "viscous_sign": ("rhs", _rhs_viscous("sign")),
    "viscous_sqrt": ("rhs", _rhs_viscous("sqrt")),
    "dft_sign": ("_unit_root_table", _roots_conj),
    "c2r_weights": ("_c2r_matrices", _c2r_no_weights),
    "idft_norm": ("idft3", _idft_missing_norm),
    "dft_axes": ("dft3", _dft_axes_swapped),
    "energy_weights": ("_hermitian_weight", _weights_flat),
    "mask_cutoff": ("dealias_mask", _mask_round),
    "kz_nyquist_sign": ("wavenumber_mesh", _mesh_kz_nyquist_negative),
    "divergence_zero": ("divergence_max", _divergence_zero),
    "divergence_transposed": ("divergence_max", _divergence_transposed),
    "point_nyquist_sign": ("idft3_point", _point_variant),
    "point_conjugate_roots": ("idft3_point", _point_forward_sign),
}


def _rk4_wrong_offset(uh, nu, dt, mesh, mask):
    def f(v):
        return spectral.rhs(v, nu, mesh, mask)
    k1 = f(uh)
    k2 = f(uh + (dt / 2) * k1)
    k3 = f(uh + dt * k2)                   # offset dt instead of dt/2
    k4 = f(uh + dt * k3)
    return uh + (dt / 6) * (k1 + 2 * k2 + 2 * k3 + k4)


def _rk4_wrong_weights(uh, nu, dt, mesh, mask):
    def f(v):
        return spectral.rhs(v, nu, mesh, mask)
    k1 = f(uh)
    k2 = f(uh + (dt / 2) * k1)
    k3 = f(uh + (dt / 2) * k2)
    k4 = f(uh + dt * k3)
    return uh + (dt / 6) * (2 * k1 + k2 + 2 * k3 + k4)    # weights of k1 and k2 swapped


MUTATIONS["rk4_stage_offset"] = ("rk4_step", _rk4_wrong_offset)
MUTATIONS["rk4_weights"] = ("rk4_step", _rk4_wrong_weights)


def _euler_half_step(uh, nu, dt, mesh, mask):
    return uh + spectral.rhs(uh, nu, mesh, mask) * (0.5 * dt)


MUTATIONS["euler_half_step"] = ("euler_step", _euler_half_step)


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name, monkeypatch):
    attr, fn = MUTATIONS[name]
    monkeypatch.setattr(spectral, attr, fn)
    failures = pins.fast_pin_failures()
    assert failures, f"planted mistake {name} passed every fast pin"
