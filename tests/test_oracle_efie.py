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


def _touching_rwg_pairs(rwg):
    """(m, n) with m != n whose supports share at least one vertex."""
    T = rwg["T"]
    verts = [set(T[rwg["tp"][m]]) | set(T[rwg["tm"][m]]) for m in range(rwg["N"])]
    return np.array([(m, n) for m in range(rwg["N"]) for n in range(rwg["N"])
                     if m != n and verts[m] & verts[n]])


def test_singular_entries_converge_with_order(ico):
    """Self and adjacent entries (singularity subtraction) converge as the outer
    rule order rises (4 -> 8 -> 12 collapsed Gauss, against 16); Radon-7 is within
    a few percent of the converged values."""
    rwg = ico(1)
    k = 2.0
    Zs = {n: cfill.fill(rwg, k, rule=collapsed_gauss(n)) for n in (4, 8, 12, 16)}
    Z7 = cfill.fill(rwg, k)
    diag = np.arange(rwg["N"])
    adj = _touching_rwg_pairs(rwg)
    assert len(adj) > 10 * rwg["N"]
    for rows, cols in ((diag, diag), (adj[:, 0], adj[:, 1])):
        ref = Zs[16][rows, cols]
        scale = np.max(np.abs(ref))
        err = {n: np.max(np.abs(Zs[n][rows, cols] - ref)) / scale for n in (4, 8, 12)}
        assert err[12] < err[8] < err[4], err
        assert err[8] < 5e-3 and err[12] < 1e-3, err
        e7 = np.max(np.abs(Z7[rows, cols] - ref)) / scale
        assert e7 < 0.05, e7


def test_touching_pairs_converge_and_orderings_agree(ico):
    """Triangle pairs that touch (p = q, a shared edge, a shared vertex): the
    singularity-subtracted blocks converge with the outer order (each doubling of
    the collapsed-Gauss order gains at least a factor 4), and the two orderings of
    the static part, p outer / q inner and q outer / p inner (equal in exact
    integration), approach each other: the un-averaged asymmetry shrinks with the
    outer order."""
    rwg = ico(1)
    k = 2.0
    T = rwg["T"]
    sets = [set(t) for t in T]
    classes = {"self": [], "edge": [], "vertex": []}
    for p in range(rwg["F"]):
        for q in range(rwg["F"]):
            n = len(sets[p] & sets[q])
            key = "self" if p == q else {2: "edge", 1: "vertex"}.get(n)
            if key:
                classes[key].append((p, q))
    rules = {n: efie.Geometry(rwg, collapsed_gauss(n)) for n in (4, 8, 16, 32)}
    G7 = efie.Geometry(rwg)
    for key, pairs in classes.items():
        assert pairs, key
        for p, q in pairs[::max(1, len(pairs) // 8)]:
            vals = {n: efie.singular_block(G, p, q, k, orderings=True) for n, G in rules.items()}
            J32, J032 = vals[32][0], vals[32][1]

            def err(J, J0):
                return max(np.max(np.abs(J - J32)) / np.max(np.abs(J32)), abs(J0 - J032) / abs(J032))

            def asym(v):
                (a, a0), (b, b0) = v[2]
                return max(np.max(np.abs(a - b)), abs(a0 - b0)) / max(np.max(np.abs(v[0])), abs(v[1]))

            e = {n: err(vals[n][0], vals[n][1]) for n in (4, 8, 16)}
            s = {n: asym(vals[n]) for n in (4, 8, 16, 32)}
            assert e[8] < 0.25 * e[4] and e[16] < 0.25 * e[8], (key, p, q, e)
            assert e[16] < 1e-4, (key, p, q, e)
            assert s[32] < s[16] < s[8] < s[4], (key, p, q, s)
            J7, J07, _ = efie.singular_block(G7, p, q, k, orderings=True)
            assert err(J7, J07) < 0.02, (key, p, q, err(J7, J07))


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
