"""Seeded random isotropic initial condition, plain FP64 NumPy.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's own initial condition is the Taylor-Green vortex (Sec. 4.2,
Appendix); this random solenoidal field is a synthetic workload for the
larger runs and the ensemble.  Recipe, per half-spectrum mode (ix, iy, iz)
and component c of a grid of size N:

1. counter key = (seed << 40) XOR (((c N + ix) N + iy)(N/2+1) + iz); two
   uniforms u1, u2 in (0, 1] from the SplitMix64 output function applied to
   2 key and 2 key + 1 (Steele, Lea & Flood, OOPSLA 2014): the output for
   counter x is mix(x + 0x9E3779B97F4A7C15), and a 64-bit output z becomes
   ((z >> 11) + 1) * 2^-53;
2. Box-Muller: g = sqrt(-2 ln u1) (cos 2 pi u2 + i sin 2 pi u2) / sqrt(2);
3. project onto divergence-free: g -= k (k . g) / |k|^2;
4. amplitude: u_hat = g sqrt(E(|k|) / (4 pi |k|^2)) N^3 with
   E(k) = k^4 exp(-2 (k/k0)^2); zero at k = 0 and outside the dealias mask;
5. Hermitian planes kz = 0 and kz = N/2: a mode whose mirror
   ((-ix) mod N, (-iy) mod N) precedes it in (iy, ix) lexicographic order
   takes the conjugate of its mirror's value; a self-mirrored mode keeps only
   its real part.  (Every mirror value is recomputed from its own counters.)
6. scale the whole field so that E = 0.5 exactly (E as in spectral.energy).

Parity: pinned by published SplitMix64 outputs, by the invariants the recipe
guarantees (E = 0.5, divergence-free, Hermitian planes, masked), and by the
shell spectrum shape on a large grid.
"""
import numpy as np

from .spectral import dealias_mask, energy, project, wavenumber_mesh

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(x):
    """SplitMix64 output function for counter array x (uint64):
    z = x + gamma; z = (z ^ z>>30) * M1; z = (z ^ z>>27) * M2; z ^ z>>31."""
    z = np.asarray(x, dtype=np.uint64) + _GAMMA
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def splitmix64_stream(seed, n):
    """The first n outputs of a SplitMix64 generator whose state starts at
    seed: output j (j = 1..n) is the output function of seed + (j-1) gamma."""
    j = np.arange(n, dtype=np.uint64)
    return splitmix64(np.uint64(seed) + j * _GAMMA)


def _unit(z):
    """53-bit double in (0, 1] from a 64-bit SplitMix64 output."""
    return ((z >> np.uint64(11)).astype(np.float64) + 1.0) * 2.0 ** -53


def _gaussian_field(N, seed):
    """Complex Gaussian g[c, ix, iy, iz] with E|g|^2 = 1 (steps 1-2)."""
    M = N // 2 + 1
    c, ix, iy, iz = np.meshgrid(np.arange(3), np.arange(N), np.arange(N),
                                np.arange(M), indexing="ij")
    idx = (((c * N + ix) * N + iy) * M + iz).astype(np.uint64)
    key = (np.uint64(seed) << np.uint64(40)) ^ idx
    u1 = _unit(splitmix64(key * np.uint64(2)))
    u2 = _unit(splitmix64(key * np.uint64(2) + np.uint64(1)))
    r = np.sqrt(-2.0 * np.log(u1))
    return (r * np.cos(2.0 * np.pi * u2) + 1j * r * np.sin(2.0 * np.pi * u2)) / np.sqrt(2.0)


def _hermitian_planes(uh):
    """Step 5 on the kz = 0 and kz = N/2 planes, in place."""
    N = uh.shape[1]
    ix = np.arange(N)[:, None]
    iy = np.arange(N)[None, :]
    mx = (-ix) % N
    my = (-iy) % N
    mirror_first = (my < iy) | ((my == iy) & (mx < ix))
    self_mirror = (mx == ix) & (my == iy)
    for iz in (0, N // 2):
        plane = uh[:, :, :, iz].copy()
        mirrored = np.conj(plane[:, mx % N, my % N])   # value at the mirror, conjugated
        out = np.where(mirror_first[None], mirrored, plane)
        out = np.where(self_mirror[None], out.real + 0j, out)
        uh[:, :, :, iz] = out
    return uh


def random_isotropic(N, seed, k0=4.0, energy_target=0.5, rule="text"):
    """Random solenoidal half-spectrum (3, N, N, N/2+1) complex128; see the
    module docstring for the exact recipe."""
    K, K2 = wavenumber_mesh(N)
    g = _gaussian_field(N, seed)
    g = project(g, K, K2)                                      # step 3
    kmag = np.sqrt(K2.astype(np.float64))
    safe = np.where(K2 == 0, 1.0, kmag)
    spec = safe ** 4 * np.exp(-2.0 * (safe / k0) ** 2)
    amp = np.sqrt(spec / (4.0 * np.pi * safe ** 2)) * float(N) ** 3
    amp = np.where((K2 == 0) | ~dealias_mask(N, rule), 0.0, amp)
    uh = g * amp                                               # step 4
    _hermitian_planes(uh)                                      # step 5
    e = energy(uh)
    return uh * np.sqrt(energy_target / e)                     # step 6
