"""Pins of the oracle's mesh / RWG table and quadrature against closed forms."""
import math

import numpy as np
import pytest

from oracle.mesh import MeshError, rwg_table, star_matrix, triangle_edges, vertex_loops
from oracle.quadrature import collapsed_gauss, radon7
from paper_2606_13482_amd.inputs import cube_sphere, icosphere


@pytest.mark.parametrize("level,area", [(2, 12.330), (4, 12.551), (5, 12.563)])
def test_icosphere_counts_and_area(level, area):
    V, T = icosphere(level)
    F = T.shape[0]
    assert F == 20 * 4 ** level
    rwg = rwg_table(V, T)
    assert rwg["N"] == 3 * F // 2
    # Euler characteristic of a sphere
    assert V.shape[0] - rwg["N"] + F == 2
    assert abs(rwg["area"].sum() - area) < 1e-3
    assert rwg["area"].sum() < 4 * math.pi
    # enclosed volume by the divergence theorem is positive (outward orientation)
    vol = np.sum(rwg["area"] * np.einsum("ij,ij->i", rwg["normal"], rwg["cent"])) / 3.0
    assert vol > 0 and abs(vol - 4 * math.pi / 3) < 0.5


@pytest.mark.parametrize("fam", ["sphere", "ellipsoid", "rounded_cube"])
def test_cube_sphere_counts(fam):
    n = 6
    V, T = cube_sphere(n, fam, axes=(1.0, 2.0, 1.5))
    assert V.shape[0] == 6 * n * n + 2 and T.shape[0] == 12 * n * n
    rwg = rwg_table(V, T)
    assert rwg["N"] == 18 * n * n


def test_rwg_conventions(ico):
    rwg = ico(1)
    T = rwg["T"]
    for m in range(rwg["N"]):
        lo, hi = rwg["edges"][m]
        assert lo < hi
        tp, tm = rwg["tp"][m], rwg["tm"][m]
        # c+ traverses lo -> hi, c- traverses hi -> lo
        cyc = lambda t, a, b: any(T[t, i] == a and T[t, (i + 1) % 3] == b for i in range(3))
        assert cyc(tp, lo, hi) and cyc(tm, hi, lo)
        assert rwg["vp"][m] not in (lo, hi) and rwg["vm"][m] not in (lo, hi)
    assert np.all(np.diff(rwg["edges"][:, 0] * 10 ** 6 + rwg["edges"][:, 1]) > 0)


def test_divergence_free_loops(ico):
    """Sigma^T L = 0 exactly: every vertex loop is divergence free (Sec. VI-A)."""
    rwg = ico(2)
    S = star_matrix(rwg)
    L = vertex_loops(rwg)
    assert np.array_equal(S.T @ L.T, np.zeros((rwg["F"], L.shape[0])))
    # stars and loops: rank(Sigma) = F - 1 on a closed surface, loops span nv - 1
    assert np.linalg.matrix_rank(S) == rwg["F"] - 1
    assert np.linalg.matrix_rank(L) == L.shape[0] - 1


def test_triangle_slots(ico):
    rwg = ico(1)
    m_of, s_of = triangle_edges(rwg)
    # every RWG appears once with +1 (on c+) and once with -1 (on c-)
    for m in range(rwg["N"]):
        hits = np.argwhere(m_of == m)
        assert hits.shape[0] == 2
        assert sorted(s_of[tuple(h)] for h in hits) == [-1.0, 1.0]


def test_mesh_errors():
    V, T = icosphere(1)
    with pytest.raises(MeshError):
        rwg_table(V, T[:-1])                       # open
    T2 = T.copy(); T2[0] = T2[0][[0, 2, 1]]
    with pytest.raises(MeshError):
        rwg_table(V, T2)                           # inconsistent orientation
    V2 = V.copy(); V2[T[0, 1]] = V2[T[0, 0]]
    with pytest.raises(MeshError):
        rwg_table(V2, T)                           # zero area


def _exact_monomial(a, b, c):
    """int over the unit reference triangle (area 1/2) of l1^a l2^b l3^c, relative to area:
    2 * a! b! c! / (a + b + c + 2)!  (Dirichlet integral)."""
    return 2.0 * math.factorial(a) * math.factorial(b) * math.factorial(c) / math.factorial(a + b + c + 2)


def test_radon_degree_five():
    bary, w = radon7()
    assert abs(w.sum() - 1.0) < 1e-15
    worst5 = 0.0
    for a in range(7):
        for b in range(7 - a):
            for c in range(7 - a - b):
                got = np.sum(w * bary[:, 0] ** a * bary[:, 1] ** b * bary[:, 2] ** c)
                err = abs(got - _exact_monomial(a, b, c))
                if a + b + c <= 5:
                    worst5 = max(worst5, err)
    assert worst5 < 1e-15
    # degree 6 is not integrated exactly
    got = np.sum(w * bary[:, 0] ** 6)
    assert abs(got - _exact_monomial(6, 0, 0)) > 1e-6


@pytest.mark.parametrize("n", [3, 5, 8])
def test_collapsed_gauss_degree(n):
    bary, w = collapsed_gauss(n)
    for a in range(2 * n - 1):
        for b in range(2 * n - 1 - a):
            c = 2 * n - 2 - a - b
            got = np.sum(w * bary[:, 0] ** a * bary[:, 1] ** b * bary[:, 2] ** c)
            assert abs(got - _exact_monomial(a, b, c)) < 1e-14


@pytest.mark.parametrize("level,fam", [(1, None), (2, None), (None, "ellipsoid")])
def test_flagged_pairs_brute_force(level, fam):
    """The flagged-pair matrix equals a pair-by-pair loop over the reading's
    definition: the triangles share a vertex (p = q included), or the squared
    centroid distance is strictly below (2 max(longest edge of p, of q))^2.  The
    loop computes areas, centroids and longest edges from the vertices itself."""
    from oracle.mesh import flagged_pairs
    if fam is None:
        V, T = icosphere(level)
    else:
        V, T = cube_sphere(4, fam, axes=(1.0, 1.7, 2.4))
    rwg = rwg_table(V, T)
    got = flagged_pairs(rwg, 2.0)
    F = T.shape[0]
    cent = [sum(V[v] for v in t) / 3.0 for t in T]
    longest = [max(math.dist(V[t[a]], V[t[(a + 1) % 3]]) for a in range(3)) for t in T]
    n_touch = n_near = 0
    for p in range(F):
        for q in range(F):
            touch = len(set(T[p]) & set(T[q])) > 0
            d2 = sum((cent[p][c] - cent[q][c]) ** 2 for c in range(3))
            thr = 2.0 * max(longest[p], longest[q])
            want = touch or d2 < thr * thr
            n_touch += touch
            n_near += want and not touch
            assert got[p, q] == want, (p, q)
    assert n_touch > 10 * F and n_near > 0
