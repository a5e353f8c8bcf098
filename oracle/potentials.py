"""Closed-form integrals of 1/R and (y - x)/R over a flat triangle (oracle).

The paper does not treat singular integrals.  The reading is singularity
subtraction with the static kernel integrated in closed form over the source
triangle (Wilton, Rao, Glisson, Schaubert, Butler, IEEE TAP 32(3), 1984;
Graglia, IEEE TAP 41(10), 1993).  Derivation restated here:

For an observation point x and a triangle with unit normal n, let
h = n.(x - a) (a any vertex) and rho = x - h n the projection of x onto the
plane.  For each edge P -> Q (counter-clockwise about n):
    l = (Q - P)/|Q - P|,   u = l x n           (outward in-plane edge normal)
    l+ = (Q - rho).l,  l- = (P - rho).l,  P0 = (P - rho).u
    R0^2 = P0^2 + h^2,  R+- = sqrt(R0^2 + l+-^2)
    f    = ln((R+ + l+)/(R- + l-))   (= ln((R- - l-)/(R+ - l+)), used when l+ + l- < 0)
    beta = atan(P0 l+/(R0^2 + |h| R+)) - atan(P0 l-/(R0^2 + |h| R-))
Then
    K0(x) = int 1/R dS      = sum_edges [P0 f - |h| beta]
    K1(x) = int (y - x)/R dS = 1/2 sum_edges u [R0^2 f + l+ R+ - l- R-] - h n K0
The in-plane part of K1 is the divergence theorem applied to grad_s R =
(rho' - rho)/R, with int R dl over an edge equal to the bracket / 2.
When R0 = 0 (x on an edge line) the f-terms are multiplied by zero and omitted.
"""
from __future__ import annotations

import numpy as np


def k0_k1(x: np.ndarray, tri: np.ndarray):
    """x: (P,3) observation points, tri: (3,3) triangle vertices (CCW about its normal).

    Returns K0 (P,) and K1 (P,3)."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    A, B, C = tri
    n = np.cross(B - A, C - A)
    n = n / np.linalg.norm(n)
    h = (x - A) @ n                                   # (P,)
    rho = x - h[:, None] * n[None, :]
    ah = np.abs(h)
    K0 = np.zeros(x.shape[0])
    K1p = np.zeros((x.shape[0], 3))
    for P, Q in ((A, B), (B, C), (C, A)):
        L = Q - P
        l = L / np.linalg.norm(L)
        u = np.cross(l, n)
        lp = (Q - rho) @ l
        lm = (P - rho) @ l
        P0 = (P - rho) @ u
        R0s = P0 * P0 + h * h
        Rp = np.sqrt(R0s + lp * lp)
        Rm = np.sqrt(R0s + lm * lm)
        with np.errstate(divide="ignore", invalid="ignore"):
            f_pos = np.log((Rp + lp) / (Rm + lm))
            f_neg = np.log((Rm - lm) / (Rp - lp))
        f = np.where(lp + lm < 0, f_neg, f_pos)
        f = np.where(R0s > 0, f, 0.0)
        with np.errstate(divide="ignore", invalid="ignore"):
            beta = (np.arctan2(P0 * lp, R0s + ah * Rp) - np.arctan2(P0 * lm, R0s + ah * Rm))
        beta = np.where(ah > 0, beta, 0.0)
        K0 += np.where(R0s > 0, P0 * f, 0.0) - ah * beta
        K1p += 0.5 * u[None, :] * (np.where(R0s > 0, R0s * f, 0.0) + lp * Rp - lm * Rm)[:, None]
    K1 = K1p - (h * K0)[:, None] * n[None, :]
    return K0, K1


def solid_angle(x: np.ndarray, tri: np.ndarray) -> np.ndarray:
    """Unsigned solid angle subtended by the triangle at points x
    (Van Oosterom and Strackee, IEEE TBME 30(2), 1983)."""
    x = np.atleast_2d(x)
    a = tri[0][None, :] - x; b = tri[1][None, :] - x; c = tri[2][None, :] - x
    la, lb, lc = (np.linalg.norm(v, axis=1) for v in (a, b, c))
    num = np.einsum("ij,ij->i", a, np.cross(b, c))
    den = (la * lb * lc + np.einsum("ij,ij->i", a, b) * lc
           + np.einsum("ij,ij->i", a, c) * lb + np.einsum("ij,ij->i", b, c) * la)
    return np.abs(2.0 * np.arctan2(num, den))
