"""Helpers for the GPU parity tests: numpy <-> device tensors and error norms."""
import sys

import numpy as np


def note(msg):
    """Print and flush what names the case before each GPU step."""
    print(msg, flush=True)
    sys.stdout.flush()


def torch_mod():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a visible GPU")
    return torch


def to_dev(a, dtype):
    torch = torch_mod()
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype == "f32":
        t = t.to(torch.complex64 if np.iscomplexobj(a) else torch.float32)
    return t.cuda().contiguous()


def to_host(t):
    return t.detach().cpu().numpy().astype(np.complex128 if t.is_complex() else np.float64)


def rel_l2(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def spectral_rel_l2(a, b):
    """Relative L2 over the half spectrum with Hermitian weights, equal to the
    physical-space relative L2 by Parseval."""
    N = a.shape[1]
    w = np.full(N // 2 + 1, 2.0)
    w[0] = w[-1] = 1.0
    num = np.sum(w * np.abs(a - b) ** 2)
    den = np.sum(w * np.abs(b) ** 2)
    return float(np.sqrt(num / den))


def embed_low_modes(N, kxy, kz):
    """Index arrays selecting the modes with wavenumbers kxy (x, y) and kz
    from an (3, N, N, N/2+1) array."""
    ix = np.where(kxy < 0, kxy + N, kxy)
    return np.ix_(range(3), ix, ix, kz)


def band_limited_spectrum(n_small, seed, kb):
    """Seeded random solenoidal half spectrum at n_small^3 (the oracle's
    random isotropic field) with every mode that has some |k_i| > kb set to
    zero.  Products of two such fields have |k_i| <= 2 kb, so while
    2 kb < n_small / 3 every size n >= n_small represents u, omega, u x omega
    and the dealiased right-hand side exactly, with u_hat scaled by
    (n / n_small)^3."""
    from oracle import ic, spectral
    uh = ic.random_isotropic(n_small, seed, k0=4.0)
    kx, _, kz = spectral.wavenumbers(n_small)
    keep = (np.abs(kx)[:, None, None] <= kb) & (np.abs(kx)[None, :, None] <= kb) & (kz[None, None, :] <= kb)
    return uh * keep


def box_index(n, kb, torch=None):
    """Index arrays (ix, iy, iz) of the modes with |k_i| <= kb in a
    (3, n, n, n/2+1) array, as a tuple usable with numpy or torch tensors."""
    k = np.concatenate([np.arange(0, kb + 1), np.arange(-kb, 0)])
    ix = np.where(k < 0, k + n, k)
    iz = np.arange(0, kb + 1)
    if torch is not None:
        ix = torch.as_tensor(ix, device="cuda")
        iz = torch.as_tensor(iz, device="cuda")
        return ix[:, None, None], ix[None, :, None], iz[None, None, :]
    return np.ix_(ix, ix, iz)


def embed_on_device(uh_small, n, dtype, kb):
    """The box |k_i| <= kb of uh_small (3, m, m, m/2+1) placed into a zero
    (3, n, n, n/2+1) device tensor, scaled by (n/m)^3."""
    torch = torch_mod()
    m = uh_small.shape[1]
    cdt = torch.complex128 if dtype == "f64" else torch.complex64
    out = torch.zeros((3, n, n, n // 2 + 1), dtype=cdt, device="cuda")
    box = uh_small[(slice(None),) + box_index(m, kb)] * (float(n) / m) ** 3
    bi = box_index(n, kb, torch)
    for c in range(3):
        out[c][bi] = torch.from_numpy(np.ascontiguousarray(box[c])).to(cdt).cuda()
    return out


def radix_plan(s, rs):
    """Variant indices of the solver's current plan with every pass that has a
    variant of radix plan rs at its current shape switched to it, and the
    passes switched."""
    var, plan = s.plan_variants_ex(), s.plan_ex()
    moved = []
    for p, i in plan.items():
        cur = var[p][i]
        keys = ("width", "xcd_pair", "y_elems", "curl_in_y")
        hit = [j for j, d in enumerate(var[p]) if d["radix"] == rs and all(d[k] == cur[k] for k in keys)]
        if hit:
            plan[p] = hit[0]
            moved.append(p)
    return plan, moved
