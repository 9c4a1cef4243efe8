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
