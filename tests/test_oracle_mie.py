"""Mie series pins and method-of-moments convergence towards it."""
import math

import numpy as np
import pytest

from oracle import cfill, efie, krylov, mie
from oracle.mesh import rwg_table
from paper_2606_13482_amd.inputs import icosphere


def test_rayleigh_limit():
    """sigma_back / (pi a^2) -> 9 (ka)^4 for a small PEC sphere (Rayleigh)."""
    for x in (1e-3, 1e-2):
        assert abs(mie.backscatter_normalised(x) / (9 * x ** 4) - 1) < 5 * x ** 2 + 1e-9


def test_energy_conservation():
    """Lossless PEC: Q_sca = Q_ext (optical theorem)."""
    for x in (0.5, 2.0, 10.0, 20.0):
        assert abs(mie.q_sca(x) - mie.q_ext(x)) < 1e-12 * mie.q_ext(x)


def test_bistatic_integral_equals_total():
    """The bistatic RCS integrated over all directions is 4 pi sigma_total = 4 pi Q_sca pi a^2;
    this pins the angular functions and the 4 pi / k^2 normalisation."""
    k, a = 2.0, 1.0
    nt, nph = 200, 64
    t, wt = np.polynomial.legendre.leggauss(nt)
    th = np.arccos(t)
    tot = 0.0
    for j in range(nph):
        ph = 2 * math.pi * j / nph
        tot += np.sum(wt * mie.rcs(k, a, th, ph)) * 2 * math.pi / nph
    assert abs(tot / (4 * math.pi * mie.q_sca(k * a) * math.pi * a * a) - 1) < 1e-10


def test_resonance_peak_and_optical_limit():
    xs = np.linspace(0.6, 1.6, 401)
    vals = np.array([mie.backscatter_normalised(x) for x in xs])
    i = int(np.argmax(vals))
    assert 3.5 < vals[i] < 3.8 and 0.95 < xs[i] < 1.1
    # optical limit: tends to 1 (geometric optics) with decaying oscillations
    assert abs(mie.backscatter_normalised(200.0) - 1) < 0.05


def test_mom_converges_to_mie():
    """Bistatic RCS of the oracle MoM solution (LU) approaches the Mie series as
    the icosphere is refined (k = 2, radius 1, E- and H-plane cuts)."""
    k = 2.0
    th = np.linspace(0.05, math.pi - 0.05, 25)
    errs = []
    for level in (1, 2, 3):
        V, T = icosphere(level)
        rwg = rwg_table(V, T)
        Z = cfill.fill(rwg, k)
        b = efie.rhs(rwg, k, np.array([[0, 0, 1.0]]), np.array([[1.0, 0, 0]]))[0]
        x = krylov.lu_solve(Z, b)
        e_plane = np.stack([np.sin(th), 0 * th, np.cos(th)], 1)
        h_plane = np.stack([0 * th, np.sin(th), np.cos(th)], 1)
        mom = np.concatenate([efie.rcs(rwg, k, x, e_plane), efie.rcs(rwg, k, x, h_plane)])
        ref = np.concatenate([mie.rcs(k, 1.0, th, 0.0), mie.rcs(k, 1.0, th, math.pi / 2)])
        errs.append(np.sqrt(np.mean((mom - ref) ** 2) / np.mean(ref ** 2)))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 0.03
