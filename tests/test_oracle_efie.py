"""Pins of the oracle's EFIE fill: structure the paper states (Sec. II, Sec. VI-A)
and properties fixed by the mathematics (symmetry, rigid-motion invariance,
quadrature convergence)."""
import math

import numpy as np
import pytest

from oracle import cfill, efie
from oracle.mesh import rwg_table, star_matrix, vertex_loops
from oracle.quadrature import collapsed_gauss
from paper_2606_13482_amd.inputs import icosphere


def test_numpy_and_c_fill_agree(ico):
    rwg = ico(1)
    Zn = efie.fill(rwg, 2.0)
    Zc = cfill.fill(rwg, 2.0)
    assert np.max(np.abs(Zn - Zc)) / np.max(np.abs(Zn)) < 1e-14


def test_transpose_symmetry(ico):
    """Z = Z^T (Galerkin EFIE with identical test and basis functions); the
    averaged singular treatment keeps it exact up to rounding."""
    Z = cfill.fill(ico(3), 6.0)
    assert np.max(np.abs(Z - Z.T)) / np.max(np.abs(Z)) < 1e-14


def test_loop_null_space_and_star_identity(ico):
    """The scalar-potential part annihilates divergence-free loops (null space of
    T_Phi, Sec. VI-A) and equals Sigma V Sigma^T with the piecewise-constant single
    layer V (star factorisation, Sec. VI-A; sign: Z = jk T_A + (1/jk) Sigma V Sigma^T,
    i.e. T_Phi = -Sigma V Sigma^T under eq:matTPhi's sign)."""
    rwg = ico(1)
    k = 2.0
    Z, A, P = efie.fill(rwg, k, parts=True)
    L = vertex_loops(rwg).T                     # (N, nv)
    rel = np.linalg.norm(P @ L) / (np.linalg.norm(P) * np.linalg.norm(L))
    assert rel < 1e-14
    # the full matrix acts on loops through T_A only
    relz = np.linalg.norm(Z @ L - 1j * k * (A @ L)) / (np.linalg.norm(Z) * np.linalg.norm(L))
    assert relz < 1e-14
    S = star_matrix(rwg)
    Vm = efie.scalar_single_layer(rwg, k)
    assert np.max(np.abs(P - S @ Vm @ S.T)) / np.max(np.abs(P)) < 1e-14
    # and the vector part does not vanish on loops
    assert np.linalg.norm(A @ L) / (np.linalg.norm(A) * np.linalg.norm(L)) > 1e-3


def test_rigid_motion_invariance():
    V, T = icosphere(2)
    k = 3.0
    Z0 = cfill.fill(rwg_table(V, T), k)
    th = 0.7
    Rz = np.array([[math.cos(th), -math.sin(th), 0], [math.sin(th), math.cos(th), 0], [0, 0, 1.0]])
    Rx = np.array([[1.0, 0, 0], [0, math.cos(1.1), -math.sin(1.1)], [0, math.sin(1.1), math.cos(1.1)]])
    V2 = V @ (Rx @ Rz).T + np.array([0.3, -1.2, 2.5])
    Z1 = cfill.fill(rwg_table(V2, T), k)
    assert np.max(np.abs(Z1 - Z0)) / np.max(np.abs(Z0)) < 1e-12


def test_regular_quadrature_convergence(ico):
    """For separated RWG pairs the Radon-7 entries approach the converged
    high-order (collapsed Gauss) integrals; the high-order rules agree closely."""
    rwg = ico(1)
    k = 2.0
    Z7 = cfill.fill(rwg, k, singular=False)
    Z8 = cfill.fill(rwg, k, rule=collapsed_gauss(8), singular=False)
    Z12 = cfill.fill(rwg, k, rule=collapsed_gauss(12), singular=False)
    mid = 0.5 * (rwg["cent"][rwg["tp"]] + rwg["cent"][rwg["tm"]])
    d = np.linalg.norm(mid[:, None, :] - mid[None, :, :], axis=2)
    far = d > 1.2
    assert far.sum() > 1000
    ref = np.max(np.abs(Z12[far]))
    assert np.max(np.abs(Z8[far] - Z12[far])) / ref < 1e-9
    e7 = np.max(np.abs(Z7[far] - Z12[far])) / ref
    assert e7 < 2e-3


def test_singular_entries_converge_with_order(ico):
    """Self and touching entries (singularity subtraction) converge as the outer
    rule order rises; Radon-7 is within a few percent of the converged values."""
    rwg = ico(1)
    k = 2.0
    Zs = {n: cfill.fill(rwg, k, rule=collapsed_gauss(n)) for n in (4, 8, 16)}
    Z7 = cfill.fill(rwg, k)
    diag = np.arange(rwg["N"])
    d48 = np.max(np.abs(Zs[4][diag, diag] - Zs[16][diag, diag]) / np.abs(Zs[16][diag, diag]))
    d816 = np.max(np.abs(Zs[8][diag, diag] - Zs[16][diag, diag]) / np.abs(Zs[16][diag, diag]))
    assert d816 < d48 and d816 < 5e-3
    e7 = np.max(np.abs(Z7[diag, diag] - Zs[16][diag, diag]) / np.abs(Zs[16][diag, diag]))
    assert e7 < 0.05


def test_fill_rows_matches_full(ico):
    rwg = ico(2)
    Z = cfill.fill(rwg, 2.0)
    rows = np.array([0, 17, 250, 479])
    Zr = efie.fill_rows(rwg, 2.0, rows)
    assert np.max(np.abs(Zr - Z[rows])) / np.max(np.abs(Z)) < 1e-14


def test_rhs_closed_form_for_constant_field(ico):
    """For a uniform field (k -> 0 limit of the plane wave) the excitation is
    int f_m . e = e . (int f_m) and int_p (r - v_p)/(2A_p) dS = (c_p - v_p)/2 per triangle."""
    rwg = ico(2)
    e = np.array([0.3, -0.5, 0.8])
    B = efie.rhs(rwg, 1e-12, np.array([[0, 0, 1.0]]), e[None])[0]
    V = rwg["V"]
    want = 0.5 * ((rwg["cent"][rwg["tp"]] - V[rwg["vp"]]) - (rwg["cent"][rwg["tm"]] - V[rwg["vm"]])) @ e
    assert np.max(np.abs(B - want)) < 1e-12
