"""Multiplicative Calderon preconditioner of the EFIE (oracle).

TEST INFRASTRUCTURE ONLY (see the package header).

The paper applies the multiplicative Calderon preconditioner of Andriulli et
al. (IEEE TAP 56(8), 2008) in all of its simulations (Sec. VI-A, remark on the
star-split operator; Sec. VII, setup of the numerical results) without
restating it.  What is computed here, from that construction:

  * the barycentric refinement of the mesh: every triangle is cut into six by
    its centroid and its edge midpoints;
  * one Buffa-Christiansen (BC) function b_m per RWG function f_m, a
    combination of RWG functions of the refined mesh (unnormalised, as the RWG
    functions of Sec. II) supported on the dual cells of the two end vertices
    of edge m (the refined triangles touching that vertex);
  * the mixed Gram matrix G_mn = <n x b_m, f_n>;
  * the EFIE matrix in the BC basis, T_BC = C Z_b C^T, with Z_b the EFIE
    matrix of the refined mesh (same fill as the RWG matrix) and C the BC
    coefficients;
  * the preconditioner M = -G^{-1} T_BC G^{-T}.  For u = sum x_n f_n, the BC
    field w = sum y_k b_k with n x w = T u tested against the RWG functions
    has G^T y = Z x; the RWG field v = sum c_n f_n with n x v = T w tested
    against the BC functions has -G c = T_BC y (since b . (n x f) =
    -(n x b) . f).  So c = M Z x, and M Z discretises the square of the EFIE
    operator, whose spectrum accumulates at -1/4 (Calderon identity);
  * GMRES on Z M u = b, x = M u (right preconditioning, so that the GMRES
    residual is the residual of the original system, on which SCC and RSCC are
    defined).

Readings (the cited construction fixes the functions only up to choices):
  * BC function of edge m = (lo, hi): charge +1/A(hi) spread uniformly over the
    dual cell of hi (area A(hi)) and -1/A(lo) over the dual cell of lo, flux 1/2
    through each of the two refined edges that join the midpoint of m to the
    centroids of c+ and c-, and zero flux through the two halves of edge m.
    On cells of equal-area refined triangles this is the classical BC
    function; on others the charge stays exactly uniform.  The orientation
    (source at the higher vertex) makes n x b_m point along f_m, so G has a
    positive diagonal; the sign of every b_m together cancels in M.
  * refined-mesh numbering: original vertices, then edge midpoints in sorted
    edge order, then centroids; children of triangle (a, b, c) are
    (a, m_ab, g), (m_ab, b, g), (b, m_bc, g), (m_bc, c, g), (c, m_ca, g),
    (m_ca, a, g), keeping the orientation.  M does not depend on it.
"""
from __future__ import annotations

import numpy as np

from . import cfill
from .krylov import gmres
from .mesh import rwg_table


def barycentric(V: np.ndarray, T: np.ndarray):
    """Refined vertices (nv + E + F, 3), triangles (6F, 3), and per child its
    parent triangle and its corner (the one original vertex it holds)."""
    V = np.asarray(V, np.float64); T = np.asarray(T, np.int64)
    nv, F = V.shape[0], T.shape[0]
    keys = sorted({(min(int(T[t, k]), int(T[t, (k + 1) % 3])), max(int(T[t, k]), int(T[t, (k + 1) % 3])))
                   for t in range(F) for k in range(3)})
    mid = {e: nv + i for i, e in enumerate(keys)}
    E = len(keys)
    Vb = np.concatenate([V, np.array([(V[a] + V[b]) / 2 for a, b in keys]).reshape(-1, 3),
                         V[T].mean(axis=1)])
    Tb = np.empty((6 * F, 3), np.int64)
    parent = np.repeat(np.arange(F), 6)
    corner = np.empty(6 * F, np.int64)
    for t in range(F):
        g = nv + E + t
        for k in range(3):
            a, b = int(T[t, k]), int(T[t, (k + 1) % 3])
            mab = mid[(min(a, b), max(a, b))]
            Tb[6 * t + 2 * k] = (a, mab, g)
            Tb[6 * t + 2 * k + 1] = (mab, b, g)
            corner[6 * t + 2 * k], corner[6 * t + 2 * k + 1] = a, b
    return Vb, Tb, parent, corner, mid


def _rwg_on(rwgx: dict, m: int, t: int, x: np.ndarray) -> np.ndarray:
    """RWG function m of table rwgx evaluated at points x (P,3) of triangle t."""
    V = rwgx["V"]
    if t == rwgx["tp"][m]:
        return (x - V[rwgx["vp"][m]]) / (2 * rwgx["area"][t])
    assert t == rwgx["tm"][m]
    return (V[rwgx["vm"][m]] - x) / (2 * rwgx["area"][t])


def bc_coefficients(rwg: dict, Vb, Tb, corner, mid, rwgb: dict) -> np.ndarray:
    """Dense (N, N_b) matrix C: b_m = sum_e C[m, e] f^b_e (refined RWG functions)."""
    N, Nb = rwg["N"], rwgb["N"]
    nv = rwg["V"].shape[0]
    eidx = {(int(a), int(b)): i for i, (a, b) in enumerate(rwgb["edges"])}
    area_b = rwgb["area"]
    cells = [[] for _ in range(nv)]
    for t, v in enumerate(corner):
        cells[v].append(t)
    Ac = np.array([area_b[c].sum() for c in cells])

    def sigma(e, t):   # +1: f^b_e leaves t across e, -1: enters
        return 1.0 if rwgb["tp"][e] == t else -1.0

    C = np.zeros((N, Nb))
    for m in range(N):
        lo, hi = (int(v) for v in rwg["edges"][m])
        mm = mid[(lo, hi)]
        # the two halves of the dual edge: midpoint of m to the centroids of c+ and c-
        halves = [eidx[tuple(sorted((mm, int(g))))] for g in Tb[[6 * rwg["tp"][m], 6 * rwg["tm"][m]], 2]]
        # flux 1/2 out of the cell of hi through each half
        for e in halves:
            t_hi = rwgb["tp"][e] if corner[rwgb["tp"][e]] == hi else rwgb["tm"][e]
            C[m, e] = 0.5 * sigma(e, t_hi)
        for v, charge in ((hi, 1.0), (lo, -1.0)):
            cell = cells[v]
            radial = sorted({eidx[tuple(sorted((v, int(x))))] for t in cell for x in Tb[t] if x != v})
            col = {e: i for i, e in enumerate(radial)}
            A = np.zeros((len(cell) + 1, len(radial)))
            rhs = np.zeros(len(cell) + 1)
            for i, t in enumerate(cell):
                # outflow of child t: radial fluxes plus the fixed dual-edge halves
                out = 0.0
                for x in Tb[t]:
                    if x == v:
                        continue
                    e = eidx[tuple(sorted((v, int(x))))]
                    A[i, col[e]] += sigma(e, t)
                for e in halves:
                    if t in (rwgb["tp"][e], rwgb["tm"][e]):
                        out += C[m, e] * sigma(e, t)
                rhs[i] = charge * area_b[t] / Ac[v] - out
            A[-1, col[eidx[tuple(sorted((v, mm)))]]] = 1.0     # zero flux through the half of edge m
            phi, res, rank, _ = np.linalg.lstsq(A, rhs, rcond=None)
            assert rank == len(radial) and np.max(np.abs(A @ phi - rhs)) < 1e-12
            for e, i in col.items():
                C[m, e] = phi[i]
    return C


def gram(rwg: dict, rwgb: dict, C: np.ndarray, parent: np.ndarray) -> np.ndarray:
    """G[m, n] = int (n x b_m) . f_n over the surface, exactly (3-point edge-midpoint
    rule on each refined triangle, exact for the quadratic integrand)."""
    N = rwg["N"]
    Tb, Vb = rwgb["T"], rwgb["V"]
    # RWG functions of each original triangle
    owners = [[] for _ in range(rwg["F"])]
    for n in range(N):
        owners[rwg["tp"][n]].append(n)
        owners[rwg["tm"][n]].append(n)
    G = np.zeros((N, N))
    for m in range(N):
        for e in np.nonzero(C[m])[0]:
            for t in (rwgb["tp"][e], rwgb["tm"][e]):
                P = Vb[Tb[t]]
                x = (P + np.roll(P, -1, axis=0)) / 2                  # edge midpoints of the child
                nb = np.cross(Vb[Tb[t, 0]] - Vb[Tb[t, 2]], Vb[Tb[t, 1]] - Vb[Tb[t, 2]])
                nb /= np.linalg.norm(nb)
                rb = np.cross(nb, _rwg_on(rwgb, e, t, x))             # n x f^b_e
                T = parent[t]
                for n in owners[T]:
                    G[m, n] += C[m, e] * rwgb["area"][t] / 3 * np.sum(rb * _rwg_on(rwg, n, T, x))
    return G


def build(V, T, k: float):
    """Everything the preconditioner needs: dict with rwg, refined mesh and its
    table, C, G, T_BC and M (dense)."""
    rwg = rwg_table(V, T)
    Vb, Tb, parent, corner, mid = barycentric(V, T)
    rwgb = rwg_table(Vb, Tb)
    C = bc_coefficients(rwg, Vb, Tb, corner, mid, rwgb)
    G = gram(rwg, rwgb, C, parent)
    Zb = cfill.fill(rwgb, k)
    Tbc = C @ Zb @ C.T
    A1 = np.linalg.solve(G, Tbc)                        # G^{-1} T_BC
    M = -np.linalg.solve(G, A1.T).T                     # -(G^{-1} T_BC) G^{-T}
    return dict(rwg=rwg, Vb=Vb, Tb=Tb, parent=parent, corner=corner, rwgb=rwgb, C=C, G=G, Tbc=Tbc, M=M)


def gmres_right(Z: np.ndarray, M: np.ndarray, b: np.ndarray, **kw):
    """GMRES on Z M u = b; returns x = M u and the statistics (the residual of
    Z M u is the residual b - Z x of the original system)."""
    u, st = gmres(Z @ M, b, **kw)
    return M @ u, st
