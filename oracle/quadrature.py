"""Quadrature rules on triangles (oracle).

The paper only says "numerical quadrature"; the reading used here is Radon's
7-point rule of degree 5 on both triangles of a pair (Radon 1948; tabulated
in Stroud, Approximate Calculation of Multiple Integrals, 1971, rule T2:5-1).

Rules are returned as (bary (n,3), w (n,)) with weights relative to the
triangle area (summing to 1):  int_T f dA  ~=  A * sum_i w_i f(x_i).
"""
from __future__ import annotations

import math

import numpy as np


def radon7():
    """Radon's degree-5 rule: the centroid plus two orbits of 3 points.

    Orbit points are (a, a, 1-2a) and permutations with a = (6 -+ sqrt15)/21.
    Weights: 9/40 at the centroid, (155 -+ sqrt15)/1200 on the orbits."""
    s15 = math.sqrt(15.0)
    a = (6.0 - s15) / 21.0
    b = (6.0 + s15) / 21.0
    wa = (155.0 - s15) / 1200.0
    wb = (155.0 + s15) / 1200.0
    bary = [(1 / 3, 1 / 3, 1 / 3),
            (a, a, 1 - 2 * a), (a, 1 - 2 * a, a), (1 - 2 * a, a, a),
            (b, b, 1 - 2 * b), (b, 1 - 2 * b, b), (1 - 2 * b, b, b)]
    w = [9.0 / 40.0, wa, wa, wa, wb, wb, wb]
    return np.array(bary, dtype=np.float64), np.array(w, dtype=np.float64)


def collapsed_gauss(n: int):
    """Conical-product (Duffy-collapsed) Gauss rule with n*n points.

    (s,t) in [0,1]^2 -> barycentric (s, t(1-s), (1-s)(1-t)), Jacobian 2(1-s)
    relative to area.  Exact for polynomials of total degree <= 2n-2."""
    x, w = np.polynomial.legendre.leggauss(n)
    x = 0.5 * (x + 1.0)
    w = 0.5 * w
    bary, wt = [], []
    for i in range(n):
        for j in range(n):
            s, t = x[i], x[j]
            bary.append((s, t * (1 - s), (1 - s) * (1 - t)))
            wt.append(2.0 * (1 - s) * w[i] * w[j])
    return np.array(bary), np.array(wt)


def points(V: np.ndarray, T: np.ndarray, bary: np.ndarray) -> np.ndarray:
    """Quadrature points of every triangle: (F, n, 3)."""
    A = V[T[:, 0]]; B = V[T[:, 1]]; C = V[T[:, 2]]
    return (bary[None, :, 0:1] * A[:, None, :] + bary[None, :, 1:2] * B[:, None, :]
            + bary[None, :, 2:3] * C[:, None, :])
