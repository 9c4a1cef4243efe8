"""Resolution independence of the early Taylor-Green evolution: while the
energy cascade has not reached the dealias cutoff, the Fourier coefficients
u_hat / N^3 of the same run on two grids agree to rounding.  This is what
lets a 64^3 oracle run stand in for the 256^3 and 512^3 GPU runs."""
import os

import numpy as np

import workloads
from oracle import spectral

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _low(uh, kmax):
    N = uh.shape[1]
    kx, _, kz = spectral.wavenumbers(N)
    order = np.argsort(kx)
    ix = order[np.abs(kx[order]) <= kmax]
    iz = np.where(kz <= kmax)[0]
    return uh[np.ix_(range(3), ix, ix, iz)] / float(N) ** 3


def test_tg_low_modes_agree_across_grids():
    nu, dt, n = 1.0 / 1600, 1e-3, 10
    a = spectral.Solver(32, nu, dt).set_velocity(workloads.taylor_green(32)).step(n)
    b = spectral.Solver(64, nu, dt).set_velocity(workloads.taylor_green(64)).step(n)
    la, lb = _low(a.uh, 8), _low(b.uh, 8)
    assert np.max(np.abs(la - lb)) < 1e-15
    assert abs(a.energy() - b.energy()) < 1e-16
    assert abs(a.enstrophy() - b.enstrophy()) < 1e-15


def test_golden_fixture_matches_oracle_start():
    g = np.load(os.path.join(GOLDEN, "tg_re1600_n64.npz"))
    assert abs(g["energy"][0] - 0.125) < 1e-16 and abs(g["enstrophy"][0] - 0.375) < 1e-15
    # energy budget holds along the stored history: dE/dt = -2 nu Omega
    E, W, dt, nu = g["energy"], g["enstrophy"], float(g["dt"]), float(g["nu"])
    res = np.abs((E[1:] - E[:-1]) / dt + nu * (W[1:] + W[:-1]))
    assert res.max() < 1e-9
