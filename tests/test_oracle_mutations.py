"""Plant plausible mistakes in the CPU oracle and check that the pins catch
each one: evidence that the pins constrain every part of the oracle
(transforms, curl, cross product, mask, projection, viscous term, RK4,
forward Euler, diagnostics).  Mistakes are planted on the CPU only, by monkeypatching."""
import numpy as np
import pytest

import oracle_pins as pins
from oracle import spectral

_orig = {name: getattr(spectral, name) for name in (
    "cross", "curl_hat", "rhs", "dft3", "idft3", "_unit_root_table",
    "_c2r_matrices", "_hermitian_weight", "wavenumber_mesh", "dealias_mask")}


def _cross_swapped(a, b):
    return _orig["cross"](b, a)


def _curl_neg(uh, K):
    return -_orig["curl_hat"](uh, K)


def _curl_index_slip(uh, K):
    w = _orig["curl_hat"](uh, K)
    w[0] = 1j * (K[1] * uh[2] - K[2] * uh[0])
    return w


def _rhs_variant(kind):
    def rhs(uh, nu, mesh, mask):
        K, K2, K_over_K2 = mesh
        u = spectral.idft3(uh)
        w = spectral.idft3(spectral.curl_hat(uh, K))
        nh = spectral.dft3(spectral.cross(u, w))
        if kind != "no_mask":
            nh *= mask
        p_hat = np.sum(nh * K_over_K2, axis=0)
        if kind == "no_projection":
            pass
        elif kind == "projection_sign":
            nh += p_hat * K
        elif kind == "projection_transposed":
            nh -= p_hat * K[::-1]
        else:
            nh -= p_hat * K
        if kind == "viscous_sign":
            nh += nu * K2 * uh
        elif kind == "viscous_sqrt":
            nh -= nu * np.sqrt(K2) * uh
        else:
            nh -= nu * K2 * uh
        return nh
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
    K, K2, K_over_K2 = _orig["wavenumber_mesh"](N)
    K = K.copy()
    K[2, :, :, -1] *= -1
    K_over_K2 = K.astype(float) / np.where(K2 == 0, 1, K2).astype(float)
    return K, K2, K_over_K2


def _mask_round(N, rule="text"):
    kx, ky, kz = spectral.wavenumbers(N)
    lim = N / 3.0 + 1
    return (np.abs(kx)[:, None, None] < lim) & (np.abs(ky)[None, :, None] < lim) & (np.abs(kz)[None, None, :] < lim)


MUTATIONS = {
    "cross_swapped": ("cross", _cross_swapped),
    "curl_negated": ("curl_hat", _curl_neg),
    "curl_index_slip": ("curl_hat", _curl_index_slip),
    "no_mask": ("rhs", _rhs_variant("no_mask")),
    "no_projection": ("rhs", _rhs_variant("no_projection")),
    "projection_sign": ("rhs", _rhs_variant("projection_sign")),
    "projection_transposed": ("rhs", _rhs_variant("projection_transposed")),
    "viscous_sign": ("rhs", _rhs_variant("viscous_sign")),
    "viscous_sqrt": ("rhs", _rhs_variant("viscous_sqrt")),
    "dft_sign": ("_unit_root_table", _roots_conj),
    "c2r_weights": ("_c2r_matrices", _c2r_no_weights),
    "idft_norm": ("idft3", _idft_missing_norm),
    "dft_axes": ("dft3", _dft_axes_swapped),
    "energy_weights": ("_hermitian_weight", _weights_flat),
    "mask_cutoff": ("dealias_mask", _mask_round),
    "kz_nyquist_sign": ("wavenumber_mesh", _mesh_kz_nyquist_negative),
}


def _rk4_wrong_b(uh, nu, dt, mesh, mask):
    U0 = uh.copy()
    U1 = uh.copy()
    cur = uh
    for s in range(4):
        R = spectral.rhs(cur, nu, mesh, mask)
        if s < 3:
            cur = U0 + (0.5, 0.5, 0.5)[s] * dt * R
        U1 += spectral.RK4_A[s] * dt * R
    return U1


MUTATIONS["rk4_stage_offset"] = ("rk4_step", _rk4_wrong_b)


def _euler_half_step(uh, nu, dt, mesh, mask):
    return uh + spectral.rhs(uh, nu, mesh, mask) * (0.5 * dt)


MUTATIONS["euler_half_step"] = ("euler_step", _euler_half_step)


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name, monkeypatch):
    attr, fn = MUTATIONS[name]
    monkeypatch.setattr(spectral, attr, fn)
    failures = pins.fast_pin_failures()
    assert failures, f"planted mistake {name} passed every fast pin"
