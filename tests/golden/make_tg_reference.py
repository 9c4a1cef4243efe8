"""Write tg_re1600_n64.npz: the CPU oracle's Taylor-Green run at N = 64,
nu = 1/1600, dt = 1e-3 (the Re = 1600 case of Sec. 4.2), FP64.

Stored: energy and enstrophy after each of 100 steps (index 0 = initial
state), the resolution-independent Fourier coefficients u_hat / N^3 of all
modes with |k_i| <= KMAX after 10 and 50 steps, and the relative L2 norm of
the modes outside that box at those steps (the part of the field the stored
modes leave out).  While the cascade has
not reached the 64^3 dealias cutoff these equal the coefficients of the same
run on any finer grid (checked by tests/test_oracle_resolution.py), so they
serve as reference values for the 256^3 and 512^3 GPU runs.

Calls only the oracle.  Run from the repository root:
    python tests/golden/make_tg_reference.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import spectral  # noqa: E402
import workloads  # noqa: E402

N, NU, DT, STEPS, KMAX = 64, 1.0 / 1600, 1e-3, 100, 12
SNAP = (10, 50)


def low_modes(uh, N, kmax):
    kx, _, kz = spectral.wavenumbers(N)
    ix = np.where(np.abs(kx) <= kmax)[0]
    iz = np.where(kz <= kmax)[0]
    return uh[np.ix_(range(3), ix, ix, iz)] / float(N) ** 3, kx[ix], kz[iz]


def outside_fraction(uh, N, kmax):
    """Relative L2 (Hermitian-weighted, i.e. physical-space) norm of the modes
    with some |k_i| > kmax: how much of the field the stored modes leave out."""
    kx, _, kz = spectral.wavenumbers(N)
    inside = (np.abs(kx)[:, None, None] <= kmax) & (np.abs(kx)[None, :, None] <= kmax) & (kz[None, None, :] <= kmax)
    w = np.full(N // 2 + 1, 2.0)
    w[0] = w[-1] = 1.0
    a = w * np.abs(uh) ** 2
    return float(np.sqrt(np.sum(a[:, ~inside]) / np.sum(a)))


def main():
    s = spectral.Solver(N, NU, DT).set_velocity(workloads.taylor_green(N))
    E, W, snaps, outside = [s.energy()], [s.enstrophy()], {}, {}
    for n in range(1, STEPS + 1):
        s.step(1)
        E.append(s.energy())
        W.append(s.enstrophy())
        if n in SNAP:
            snaps[n], kxy, kz = low_modes(s.uh, N, KMAX)
            outside[n] = outside_fraction(s.uh, N, KMAX)
    out = os.path.join(HERE, "tg_re1600_n64.npz")
    np.savez(out, N=N, nu=NU, dt=DT, kmax=KMAX, energy=np.array(E), enstrophy=np.array(W),
             kxy=kxy, kz=kz, snap_steps=np.array(SNAP),
             **{f"modes_{n}": snaps[n] for n in SNAP},
             **{f"outside_rel_l2_{n}": outside[n] for n in SNAP})
    print("wrote", out)


if __name__ == "__main__":
    main()
