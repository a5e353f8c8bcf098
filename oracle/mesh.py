"""RWG table of a closed triangle mesh (oracle).

Follows Sec. II (Galerkin RWG basis, edge-length normalisation omitted) and
the RWG sketch of Sec. VI-A (one function per interior edge, supported on the
two triangles c+ and c- sharing the edge, free vertices x+ and x-).

Conventions (readings where the paper only draws a figure):
  * one unknown per undirected edge; edges sorted lexicographically by
    (lower vertex index, higher vertex index);
  * c+ is the triangle that traverses the edge from the lower to the higher
    vertex index (CCW seen from outside), c- the other one;
  * f_m(r) = (r - x+)/(2 A+) on c+ and (x- - r)/(2 A-) on c-, so that
    div f_m = +1/A+ on c+ and -1/A- on c-.
"""
from __future__ import annotations

import numpy as np


class MeshError(ValueError):
    pass


def triangle_geometry(V: np.ndarray, T: np.ndarray):
    """Areas (F,), unit normals (F,3), centroids (F,3), longest edge (F,)."""
    a, b, c = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
    cr = np.cross(b - a, c - a)
    twice = np.linalg.norm(cr, axis=1)
    area = 0.5 * twice
    with np.errstate(invalid="ignore", divide="ignore"):
        normal = cr / twice[:, None]
    cent = (a + b + c) / 3.0
    longest = np.max(np.stack([np.linalg.norm(b - a, axis=1), np.linalg.norm(c - b, axis=1),
                               np.linalg.norm(a - c, axis=1)], axis=1), axis=1)
    return area, normal, cent, longest


def rwg_table(V: np.ndarray, T: np.ndarray) -> dict:
    """Build the RWG table and validate the mesh.

    Returns a dict with
      edges  (N,2) int  lower, higher vertex index
      tp, tm (N,)  int  triangle c+ and c-
      vp, vm (N,)  int  free vertex of c+ and of c-
      area, normal, cent, longest  per-triangle geometry
    Raises MeshError for open / non-manifold / inconsistently oriented meshes
    and zero-area triangles.
    """
    V = np.asarray(V, dtype=np.float64)
    T = np.asarray(T, dtype=np.int64)
    F = T.shape[0]
    if F == 0 or T.ndim != 2 or T.shape[1] != 3:
        raise MeshError("need a non-empty (F,3) triangle array")
    if T.min() < 0 or T.max() >= V.shape[0]:
        raise MeshError("vertex index out of range")
    area, normal, cent, longest = triangle_geometry(V, T)
    if not np.all(area > 0):
        raise MeshError("zero-area triangle")
    directed: dict[tuple[int, int], tuple[int, int]] = {}
    for t in range(F):
        for k in range(3):
            i, j = int(T[t, k]), int(T[t, (k + 1) % 3])
            if i == j:
                raise MeshError("degenerate triangle")
            if (i, j) in directed:
                raise MeshError("edge traversed twice in one direction (orientation or manifoldness)")
            free = int(T[t, (k + 2) % 3])
            directed[(i, j)] = (t, free)
    keys = sorted({(min(i, j), max(i, j)) for (i, j) in directed})
    N = len(keys)
    edges = np.array(keys, dtype=np.int64).reshape(-1, 2)
    tp = np.empty(N, np.int64); tm = np.empty(N, np.int64)
    vp = np.empty(N, np.int64); vm = np.empty(N, np.int64)
    for m, (lo, hi) in enumerate(keys):
        if (lo, hi) not in directed or (hi, lo) not in directed:
            raise MeshError("open mesh: boundary edge")
        tp[m], vp[m] = directed[(lo, hi)]
        tm[m], vm[m] = directed[(hi, lo)]
    if 2 * N != 3 * F:
        raise MeshError("not a closed 2-manifold")
    return dict(V=V, T=T, edges=edges, tp=tp, tm=tm, vp=vp, vm=vm,
                area=area, normal=normal, cent=cent, longest=longest, N=N, F=F)


def triangle_edges(rwg: dict):
    """Per triangle, its three RWG functions: (F,3) index m, sign s, free vertex.

    Local slot k of triangle t is the RWG whose free vertex is T[t,k]
    (i.e. the edge opposite vertex k)."""
    F = rwg["F"]; T = rwg["T"]
    m_of = -np.ones((F, 3), np.int64)
    s_of = np.zeros((F, 3), np.float64)
    for m in range(rwg["N"]):
        for t, v, s in ((rwg["tp"][m], rwg["vp"][m], 1.0), (rwg["tm"][m], rwg["vm"][m], -1.0)):
            k = int(np.nonzero(T[t] == v)[0][0])
            m_of[t, k] = m
            s_of[t, k] = s
    assert np.all(m_of >= 0)
    return m_of, s_of


def flagged_pairs(rwg: dict, near_factor: float = 2.0) -> np.ndarray:
    """Boolean (F,F) matrix of pairs that get singularity subtraction.

    A pair (p,q) is flagged if the triangles share at least one vertex
    (p == q included) or if |c_p - c_q|^2 < (near_factor * max(longest_p, longest_q))^2
    (strict inequality on the squared FP64 distance).  The paper leaves the
    singular treatment open; this is the reading used throughout."""
    T = rwg["T"]; cent = rwg["cent"]; L = rwg["longest"]
    F = rwg["F"]
    nv = rwg["V"].shape[0]
    inc = np.zeros((F, nv), dtype=np.float32)
    inc[np.repeat(np.arange(F), 3), T.reshape(-1)] = 1.0
    share = (inc @ inc.T) > 0.5          # number of shared vertices (exact small integers)
    d2 = np.sum((cent[:, None, :] - cent[None, :, :]) ** 2, axis=2)
    thr = near_factor * np.maximum(L[:, None], L[None, :])
    return share | (d2 < thr * thr)


def star_matrix(rwg: dict) -> np.ndarray:
    """Sigma (N,F): +1 at (m, c+(m)), -1 at (m, c-(m))  (Sec. VI-A, star basis)."""
    S = np.zeros((rwg["N"], rwg["F"]))
    S[np.arange(rwg["N"]), rwg["tp"]] = 1.0
    S[np.arange(rwg["N"]), rwg["tm"]] = -1.0
    return S


def vertex_loops(rwg: dict) -> np.ndarray:
    """Loop (solenoidal) vectors, one per vertex, (nv, N) with entries +-1.

    The loop around vertex v circulates through the edges incident to v; with
    unnormalised RWG functions its coefficients are +-1 and it is divergence
    free, so Sigma^T L = 0 exactly (Sec. VI-A, null space of the scalar
    potential operator)."""
    V = rwg["V"]; T = rwg["T"]; N = rwg["N"]
    Lp = np.zeros((V.shape[0], N))
    for m in range(N):
        lo, hi = rwg["edges"][m]
        # In a triangle t around vertex v (CCW order v, a, b) the two edges at v
        # are traversed v->a and b->v.  With coefficient +1 when v is the lower
        # vertex of the edge and -1 when it is the higher one, the products
        # (sign of f_m on t) * coefficient are +1 and -1: the divergence cancels.
        Lp[lo, m] = 1.0
        Lp[hi, m] = -1.0
    return Lp
