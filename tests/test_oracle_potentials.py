"""Pins of the closed-form triangle potentials K0 = int 1/R and K1 = int (y-x)/R."""
import math

import numpy as np
import pytest

from oracle import cfill
from oracle.potentials import k0_k1, solid_angle
from oracle.quadrature import collapsed_gauss

TRI = np.array([[0.0, 0.0, 0.0], [1.0, 0.1, 0.0], [0.2, 0.9, 0.1]])


def _brute(x, tri, n=300):
    bary, w = collapsed_gauss(n)
    pts = bary @ tri
    A = 0.5 * np.linalg.norm(np.cross(tri[1] - tri[0], tri[2] - tri[0]))
    d = pts[None, :, :] - x[:, None, :]
    R = np.linalg.norm(d, axis=2)
    return A * np.sum(w / R, axis=1), A * np.einsum("j,pjc->pc", w, d / R[:, :, None])


def test_against_brute_force_off_surface():
    rng = np.random.default_rng(3)
    x = rng.uniform(-1, 2, (12, 3))
    n = np.cross(TRI[1] - TRI[0], TRI[2] - TRI[0]); n /= np.linalg.norm(n)
    x += 0.2 * n * np.sign((x - TRI[0]) @ n)[:, None]      # keep away from the plane
    K0, K1 = k0_k1(x, TRI)
    B0, B1 = _brute(x, TRI)
    assert np.max(np.abs(K0 - B0) / np.abs(B0)) < 1e-11
    assert np.max(np.linalg.norm(K1 - B1, axis=1) / np.linalg.norm(B1, axis=1)) < 1e-11


def test_equilateral_centroid_closed_form():
    """int over an equilateral triangle of side a of 1/|y - c| (c the centroid) = sqrt(3) a ln(2 + sqrt(3)):
    each edge is at distance a/(2 sqrt3) and seen under +-a/2, the classical
    potential of a uniform equilateral plate at its centre."""
    for a in (1.0, 0.37):
        tri = a * np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.5, math.sqrt(3) / 2, 0.0]])
        c = tri.mean(axis=0, keepdims=True)
        K0, K1 = k0_k1(c, tri)
        assert abs(K0[0] - math.sqrt(3) * a * math.log(2 + math.sqrt(3))) < 1e-14
        assert abs(math.sqrt(3) * math.log(2 + math.sqrt(3)) - 2.2810379889028387) < 1e-15
        assert np.linalg.norm(K1) < 1e-15          # symmetric about the centroid


def test_beta_sum_is_solid_angle():
    """The atan terms of K0 sum to the solid angle: d K0 / d|h| = -Omega + O(h) is avoided
    by checking Omega directly against the Van Oosterom-Strackee formula."""
    rng = np.random.default_rng(5)
    x = rng.uniform(-0.5, 1.5, (20, 3))
    from oracle import potentials
    n = np.cross(TRI[1] - TRI[0], TRI[2] - TRI[0]); n /= np.linalg.norm(n)
    om = solid_angle(x, TRI)
    # recompute sum(beta) with the same edge quantities as k0_k1
    h = (x - TRI[0]) @ n
    rho = x - h[:, None] * n
    tot = np.zeros(x.shape[0])
    for P, Q in ((TRI[0], TRI[1]), (TRI[1], TRI[2]), (TRI[2], TRI[0])):
        l = (Q - P) / np.linalg.norm(Q - P); u = np.cross(l, n)
        lp = (Q - rho) @ l; lm = (P - rho) @ l; P0 = (P - rho) @ u
        R0s = P0 ** 2 + h ** 2
        Rp = np.sqrt(R0s + lp ** 2); Rm = np.sqrt(R0s + lm ** 2)
        tot += np.arctan2(P0 * lp, R0s + np.abs(h) * Rp) - np.arctan2(P0 * lm, R0s + np.abs(h) * Rm)
    assert np.max(np.abs(np.abs(tot) - om)) < 1e-12


def test_in_plane_interior_point():
    """Point in the plane, inside: K0 by brute force with a split at the point (3 sub-triangles)."""
    x = TRI[0] * 0.3 + TRI[1] * 0.35 + TRI[2] * 0.35
    K0, _ = k0_k1(x[None], TRI)
    tot = 0.0
    for a, b in ((TRI[0], TRI[1]), (TRI[1], TRI[2]), (TRI[2], TRI[0])):
        sub = np.array([x, a, b])
        # the collapsed rule shrinks towards barycentric slot 0 (s -> 1) with
        # Jacobian 2(1 - s), which cancels the 1/R singularity at x = slot 0
        bary, w = collapsed_gauss(60)
        pts = bary @ sub
        A = 0.5 * np.linalg.norm(np.cross(a - x, b - x))
        tot += A * np.sum(w / np.linalg.norm(pts - x, axis=1))
    assert abs(K0[0] - tot) / tot < 1e-12


def test_c_version_matches_numpy():
    rng = np.random.default_rng(9)
    x = rng.uniform(-1, 2, (50, 3))
    K0, K1 = k0_k1(x, TRI)
    C0, C1 = cfill.k0_k1(x, TRI)
    assert np.max(np.abs(K0 - C0)) < 1e-14 * np.max(np.abs(K0))
    assert np.max(np.abs(K1 - C1)) < 1e-14 * np.max(np.abs(K1))
