"""Tensor-product B-spline interpolation of the Green's function and the
single-level far field built on it (oracle, FP64).  TEST INFRASTRUCTURE ONLY:
only tests/, the entry point's smoke() and the benchmark's CPU baseline use it.

What the paper states, restated plainly:

  * Degree-p B-splines on an open, equidistant knot vector of s splines on
    [0, 1] (Sec. III-A, eq:eqknots), evaluated by the Cox-de Boor recursion.
  * Interpolation of g between the boxes of a test and a trial function
    (Sec. III-A, eq:TAfactor): with B[i, m] = b_i(x_m) the splines at the
    equispaced interpolation points, the weights are W = B^-T G B^-1, G the
    samples of g between the two point grids, so that
        [T_A]_mn ~ sum_d m_{d,m}^T W m_{d,n},   m_{d,n}[i] = int f_{n,d} b_i.
    With transformed moments m~ = B^-1 m the same value is
        sum_d m~_{d,m}^T G m~_{d,n}                              (eq:TAfactorBspline)
    and the scalar potential takes the same form with the divergence moments.
  * Buffer knots (Sec. III-B): the knot vector is extended by s_b knots of the
    same spacing on each side so that the supports of all basis functions of
    the box lie inside the enlarged interpolation domain;
    s_b = ceil(max relative protrusion / du), du = 1/(s - p).
  * Stabilisation (Sec. V-B): r interior knots next to each end of the
    equidistant knot vector are removed (r from the paper's table: 0, 0, 1, 1,
    2, 2 for p = 1..6); the stabilised splines interpolate at as many
    equispaced points; moments are taken with the equidistant splines and
    mapped to the stabilised ones by knot insertion, W_stab = S^T B_s^-T G B_s^-1 S
    (S = the insertion matrix C below).
  * Knot insertion (Sec. IV-B, Boehm's algorithm): inserting u- into the
    interval [u_k, u_k+1) gives the coefficients w-_i = a_i w_i + (1 - a_i) w_i-1
    with a_i = 1 (i <= k - p), (u- - u_i)/(u_i+p - u_i) (k - p < i <= k), 0
    (i > k).  Inserting every knot of a finer vector into the unit-coefficient
    curve of coarse spline j gives row j of the refinement matrix C:
    b_j^coarse = sum_i C[j, i] b_i^fine.
  * Error bound (Sec. V-A, eq:errorapprox):
        ||Pi f - f||_inf,B <= du^(p+1) C2^(d-1) (h/2)^(p+1) sum_k ||d_k^(p+1) f||_inf,B
    with C2 <= ||B^-1||_inf (max row sum).

Readings where the paper is silent (listed in the design doc): the interpolation
points are s' equispaced points spanning the (buffered) interpolation domain,
s' the number of (stabilised) splines, end points included; an RWG function
belongs to the box that contains the mean of its two triangle centroids; two
boxes are far when their indices differ by more than one along some axis; the
moments use the fill's Radon 7-point rule on each triangle.
"""
from __future__ import annotations

import math

import numpy as np

from .efie import Geometry, green

KNOTS_TO_REMOVE = {1: 0, 2: 0, 3: 1, 4: 1, 5: 2, 6: 2}   # paper's table, per side


# ----------------------------------------------------------------------------- 1D splines
def open_knots(n: int, p: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    """Open equidistant knot vector of n splines of degree p on [lo, hi]
    (eq:eqknots mapped to [lo, hi]): p+1 copies of each end, n-p-1 interior
    knots at spacing (hi - lo)/(n - p)."""
    if n < p + 1:
        raise ValueError("need at least p + 1 splines")
    inner = [lo + (hi - lo) * (i - p - 1) / (n - p) for i in range(p + 2, n + 1)]
    return np.array([lo] * (p + 1) + inner + [hi] * (p + 1), dtype=np.float64)


def averaged_knots(n: int, p: int) -> np.ndarray:
    """Averaged knot vector for n equispaced interpolation points on [0, 1] (eq:avgknots)."""
    inner = [(2 * i - p - 3) / (2 * (n - 1)) for i in range(p + 2, n + 1)]
    return np.array([0.0] * (p + 1) + inner + [1.0] * (p + 1), dtype=np.float64)


def remove_boundary_knots(u: np.ndarray, p: int, r: int) -> np.ndarray:
    """The knot vector with the r interior knots nearest each end removed (Sec. V-B)."""
    if r == 0:
        return u.copy()
    inner = u[p + 1:len(u) - p - 1]
    if len(inner) < 2 * r:
        raise ValueError("not enough interior knots to remove")
    return np.concatenate([u[:p + 1], inner[r:len(inner) - r], u[len(u) - p - 1:]])


def basis(u: np.ndarray, p: int, x) -> np.ndarray:
    """Values of all n = len(u) - p - 1 B-splines of degree p at the points x
    (Cox-de Boor recursion, 0/0 taken as 0); (len(x), n).  The interval ending at
    the last knot is closed on the right."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    m = len(u)
    N = np.zeros((x.size, m - 1))
    last = np.max(np.nonzero(u[1:] > u[:-1])[0])          # last non-empty knot interval
    for i in range(m - 1):
        if u[i + 1] > u[i]:
            inside = (x >= u[i]) & (x < u[i + 1])
            if i == last:
                inside |= x == u[i + 1]
            N[:, i] = inside
    for d in range(1, p + 1):
        M = np.zeros((x.size, m - 1 - d))
        for i in range(m - 1 - d):
            a = u[i + d] - u[i]
            b = u[i + d + 1] - u[i + 1]
            if a > 0:
                M[:, i] += (x - u[i]) / a * N[:, i]
            if b > 0:
                M[:, i] += (u[i + d + 1] - x) / b * N[:, i + 1]
        N = M
    return N


def sampling_matrix(u: np.ndarray, p: int, pts) -> np.ndarray:
    """B[i, m] = b_i(x_m)."""
    return basis(u, p, pts).T.copy()


def equispaced(n: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    """n equispaced points on [lo, hi], the ends exactly lo and hi."""
    if n == 1:
        return np.array([0.5 * (lo + hi)])
    t = np.array([lo + (hi - lo) * m / (n - 1) for m in range(n)])
    t[0], t[-1] = lo, hi
    return t


def insert_knot(u: np.ndarray, p: int, w: np.ndarray, ubar: float):
    """Boehm's insertion of one knot (Sec. IV-B): the knot vector and the
    coefficients of the same spline curve on it."""
    n = len(u) - p - 1
    k = int(np.searchsorted(u, ubar, side="right")) - 1          # u[k] <= ubar < u[k+1]
    wb = np.zeros(n + 1)
    for i in range(n + 1):
        if i <= k - p:
            a = 1.0
        elif i <= k:
            a = (ubar - u[i]) / (u[i + p] - u[i])
        else:
            a = 0.0
        wb[i] = (a * w[i] if i < n else 0.0) + ((1.0 - a) * w[i - 1] if i >= 1 else 0.0)
    return np.insert(u, k + 1, ubar), wb


def refinement_matrix(u_coarse: np.ndarray, u_fine: np.ndarray, p: int) -> np.ndarray:
    """C (n_coarse x n_fine) with b_j^coarse = sum_i C[j, i] b_i^fine: every knot of
    the fine vector missing from the coarse one is inserted into the curve with
    unit coefficient j (Sec. IV-B)."""
    extra = list(u_fine)
    for v in u_coarse:                                  # multiset difference
        for t, e in enumerate(extra):
            if e == v:
                del extra[t]
                break
        else:
            raise ValueError("coarse knot vector not contained in the fine one")
    n = len(u_coarse) - p - 1
    C = np.zeros((n, len(u_fine) - p - 1))
    for j in range(n):
        u, w = u_coarse.copy(), np.eye(n)[j]
        for e in sorted(extra):
            u, w = insert_knot(u, p, w, e)
        assert np.array_equal(u, np.sort(u_fine))
        C[j] = w
    return C


# ----------------------------------------------------------------------------- one box's spline space
class BoxSplines:
    """The spline spaces of one box level along one axis, in the box's parameter
    coordinate t = (x - lo) / a (the box is t in [0, 1]): the equidistant knot
    vector of s splines extended by sb buffer knots per side, its stabilised
    version with r knots removed per side, the equispaced interpolation points,
    and the map A = B_stab^-1 C from equidistant-spline moments to transformed
    stabilised moments (m~ = A m along each axis)."""

    def __init__(self, s: int, p: int, sb: int = 0, stabilise: bool = True):
        self.s, self.p, self.sb = s, p, sb
        self.du = 1.0 / (s - p)
        self.lo, self.hi = -sb * self.du, 1.0 + sb * self.du
        self.n = s + 2 * sb
        self.u_eq = open_knots(self.n, p, self.lo, self.hi)
        self.r = KNOTS_TO_REMOVE[p] if stabilise else 0
        self.u_st = remove_boundary_knots(self.u_eq, p, self.r)
        self.n_st = len(self.u_st) - p - 1
        self.t = equispaced(self.n_st, self.lo, self.hi)                # interpolation points
        self.B = sampling_matrix(self.u_st, p, self.t)                   # B[i, m] = b_i^stab(t_m)
        self.C = refinement_matrix(self.u_st, self.u_eq, p)              # stab in terms of eq
        self.A = np.linalg.solve(self.B, self.C)                         # n_st x n

    def eq_basis(self, t) -> np.ndarray:
        return basis(self.u_eq, self.p, t)


# ----------------------------------------------------------------------------- single level
def box_level(rwg: dict, a: float, origin=None):
    """Uniform boxes of side a: the box index (3 ints) of every RWG function (the
    box holding the mean of its triangle centroids), the boxes' lower corners,
    and the largest protrusion of a support beyond its box relative to a."""
    V, T = rwg["V"], rwg["T"]
    if origin is None:
        origin = V.min(axis=0) - 1e-9 * a
    c = 0.5 * (rwg["cent"][rwg["tp"]] + rwg["cent"][rwg["tm"]])
    idx = np.floor((c - origin) / a).astype(np.int64)
    lo = origin + idx * a
    prot = 0.0
    for m in range(rwg["N"]):
        pts = V[np.concatenate([T[rwg["tp"][m]], T[rwg["tm"][m]]])]
        prot = max(prot, float(np.max((lo[m] - pts) / a)), float(np.max((pts - lo[m] - a) / a)))
    return idx, lo, max(prot, 0.0), np.asarray(origin)


def buffer_knots(prot_rel: float, s: int, p: int) -> int:
    """s_b = ceil(max relative protrusion / du) (Sec. III-B)."""
    return int(math.ceil(prot_rel * (s - p) - 1e-12)) if prot_rel > 0 else 0


def moments(rwg: dict, sp: BoxSplines, a: float, lo: np.ndarray, rule=None, transformed: bool = True) -> np.ndarray:
    """Transformed moments m~ (N, 4, n_st, n_st, n_st): components d = x, y, z of
    int f_m b~ and the divergence moment int div f_m b~, with b~ the transformed
    stabilised splines of the function's box (lo: its lower corner, (N, 3)) and
    the fill's quadrature rule.  transformed=False: the moments m with the
    buffered equidistant splines themselves, (N, 4, n, n, n)."""
    G = Geometry(rwg, rule)
    N = rwg["N"]
    n = sp.n_st if transformed else sp.n
    T1 = sp.A.T if transformed else np.eye(sp.n)
    out = np.zeros((N, 4, n, n, n))
    for m in range(N):
        for t, vfree, sgn in ((rwg["tp"][m], rwg["vp"][m], 1.0), (rwg["tm"][m], rwg["vm"][m], -1.0)):
            X = G.X[t]                                              # (nq, 3)
            tt = (X - lo[m]) / a                                    # parameter coordinates
            bx = sp.eq_basis(tt[:, 0]) @ T1                         # (nq, n_st): b~ along x
            by = sp.eq_basis(tt[:, 1]) @ T1
            bz = sp.eq_basis(tt[:, 2]) @ T1
            prod = np.einsum("qi,qj,qk->qijk", bx, by, bz)          # (nq, n, n, n)
            D = X - rwg["V"][vfree]                                 # (nq, 3)
            for d in range(3):
                out[m, d] += 0.5 * sgn * np.einsum("q,qijk->ijk", G.w * D[:, d], prod)
            out[m, 3] += sgn * np.einsum("q,qijk->ijk", G.w, prod)
    return out


def grid_points(sp: BoxSplines, a: float, lo_box: np.ndarray) -> np.ndarray:
    """The box's interpolation points in space, (n_st^3, 3), index order (i, j, k)."""
    t = lo_box[None, :] + a * sp.t[:, None]
    gx, gy, gz = np.meshgrid(t[:, 0], t[:, 1], t[:, 2], indexing="ij")
    return np.stack([gx.ravel(), gy.ravel(), gz.ravel()], axis=1)


def far_pairs(box_idx: np.ndarray):
    """Distinct boxes (rows of unique indices) and the far pairs among them
    (Chebyshev distance of the indices > 1)."""
    boxes, inv = np.unique(box_idx, axis=0, return_inverse=True)
    d = np.max(np.abs(boxes[:, None, :] - boxes[None, :, :]), axis=2)
    return boxes, inv.ravel(), d > 1


def far_block(mt: np.ndarray, rows, cols, sp: BoxSplines, a: float, lo_x, lo_y, k: float) -> np.ndarray:
    """Interpolated entries Z~_mn for test functions `rows` (all in the box at
    lo_x) and trial functions `cols` (box at lo_y):
    jk sum_d m~_d,m^T G m~_d,n + (1/jk) m~_4,m^T G m~_4,n (eq:TAfactorBspline)."""
    Px, Py = grid_points(sp, a, lo_x), grid_points(sp, a, lo_y)
    R = np.linalg.norm(Px[:, None, :] - Py[None, :, :], axis=2)
    Gm = green(R, k)
    A = mt[rows].reshape(len(rows), 4, -1)
    B = mt[cols].reshape(len(cols), 4, -1)
    jk = 1j * k
    out = np.zeros((len(rows), len(cols)), np.complex128)
    for d in range(4):
        out += (jk if d < 3 else 1.0 / jk) * (A[:, d, :] @ Gm @ B[:, d, :].T)
    return out


def far_product(rwg: dict, k: float, x: np.ndarray, a: float, s: int, p: int, stabilise: bool = True,
                origin=None):
    """y = Z~_far x: the single-level far field (every pair of far boxes) of the
    RWG functions with coefficients x (N,) or (R, N); returns y and the level's
    data (boxes, far mask, splines) for checks."""
    idx, lo, prot, origin = box_level(rwg, a, origin)
    sb = buffer_knots(prot, s, p)
    if 2 * sb >= s - p:
        # the buffered domains of two boxes two apart would touch: g is not smooth there
        raise ValueError("buffer knots reach half a box: use larger boxes or more splines")
    sp = BoxSplines(s, p, sb, stabilise)
    mt = moments(rwg, sp, a, lo)
    boxes, inv, far = far_pairs(idx)
    X = np.atleast_2d(x)
    Y = np.zeros_like(X, dtype=np.complex128)
    members = [np.nonzero(inv == b)[0] for b in range(len(boxes))]
    box_lo = origin + boxes * a
    for bx in range(len(boxes)):
        rows = members[bx]
        for by in np.nonzero(far[bx])[0]:
            cols = members[by]
            Zb = far_block(mt, rows, cols, sp, a, box_lo[bx], box_lo[by], k)
            Y[:, rows] += X[:, cols] @ Zb.T
    return (Y[0] if np.ndim(x) == 1 else Y), dict(boxes=boxes, inv=inv, far=far, sb=sb, splines=sp, moments=mt,
                                                   box_lo=box_lo, members=members, prot=prot)


def far_mask(inv: np.ndarray, far: np.ndarray) -> np.ndarray:
    """(N, N) boolean: the entries (m, n) whose boxes are far apart."""
    return far[inv][:, inv]


# ----------------------------------------------------------------------------- multilevel (Sec. IV)
def restriction_matrix(u_par: np.ndarray, p: int, u_ch: np.ndarray, tol: float = 1e-12) -> np.ndarray:
    """C (n_par x n_ch) with b_j^par(x) = sum_i C[j, i] b_i^ch(x) on the child's
    interval [u_ch[0], u_ch[-1]] (Sec. IV-B): every knot of the child vector that
    the parent vector lacks is inserted into the unit-coefficient curve of parent
    spline j, the two ends up to multiplicity p + 1, and the coefficients of the
    splines of the refined vector that live on the child's interval are row j.
    Requires the parent's knots inside the interval to be child knots (nested
    spaces); knots closer than tol are taken as equal."""
    a, b = u_ch[0], u_ch[-1]
    par = [float(v) for v in u_par]
    extra = []
    inner_par = [v for v in par if a - tol < v < b + tol]
    pool = list(inner_par)
    for v in u_ch:
        for t, e in enumerate(pool):
            if abs(e - v) <= tol:
                del pool[t]
                break
        else:
            extra.append(float(v))
    # parent knots strictly inside the interval must all be child knots
    if any(a + tol < v < b - tol for v in pool):
        raise ValueError("parent knots not contained in the child's knot vector")
    n_par = len(u_par) - p - 1
    n_ch = len(u_ch) - p - 1
    C = np.zeros((n_par, n_ch))
    for j in range(n_par):
        u, w = np.array(par), np.eye(n_par)[j]
        for e in sorted(extra):
            u, w = insert_knot(u, p, w, e)
        # the child's splines: the refined splines from the first copy of a on
        k0 = int(np.nonzero(np.abs(u - a) <= tol)[0][0])
        assert np.max(np.abs(u[k0:k0 + len(u_ch)] - u_ch)) <= 10 * tol
        C[j] = w[k0:k0 + n_ch]
    return C


def level_configs(s: int, p: int, sb: int, a_leaf: float, levels: int, k: float, stabilise: bool = True):
    """Spline spaces from the leaf level (index 0) up: the parent of a level keeps
    s and takes ceil(sb / 2) buffer knots when its boxes are smaller than half a
    wavelength (Sec. IV-C), and otherwise takes 2 s - p splines (the same physical
    knot spacing) and the same sb (Sec. IV-D); there are no leaves above level 0."""
    lam = 2.0 * math.pi / k
    cfg = [BoxSplines(s, p, sb, stabilise)]
    for l in range(1, levels):
        a_par = a_leaf * 2 ** l
        prev = cfg[-1]
        if a_par < 0.5 * lam:
            cfg.append(BoxSplines(prev.s, p, -(-prev.sb // 2), stabilise))
        else:
            cfg.append(BoxSplines(2 * prev.s - p, p, prev.sb, stabilise))
    return cfg


def transfer_matrices(child: BoxSplines, parent: BoxSplines):
    """The two 1D transfer matrices (child at the lower / upper half of the
    parent): parent equidistant splines in terms of the child's, both knot
    vectors in the parent's parameter coordinate."""
    out = []
    for c in (0, 1):
        u_ch = 0.5 * c + 0.5 * child.u_eq
        out.append(restriction_matrix(parent.u_eq, parent.p, u_ch))
    return out


def apply3(A: np.ndarray, B: np.ndarray, Cm: np.ndarray, M: np.ndarray) -> np.ndarray:
    """(A (x) B (x) C) applied to the last three axes of M."""
    return np.einsum("ia,jb,kc,...abc->...ijk", A, B, Cm, M, optimize=True)


def translation_kernel(sp: BoxSplines, a: float, offset: np.ndarray, k: float) -> np.ndarray:
    """K[d] = g(|offset + h d|), d in [-(n-1), n-1]^3 (z fastest), h the spacing
    of the level's interpolation points: G_XY[i, j] = K[i - j] for boxes whose
    lower corners differ by offset (three-level Toeplitz, Sec. III-C)."""
    n = sp.n_st
    h = a * (sp.t[1] - sp.t[0]) if n > 1 else 0.0
    d = np.arange(-(n - 1), n)
    D = np.stack(np.meshgrid(d, d, d, indexing="ij"), -1)
    R = np.linalg.norm(offset[None, None, None, :] + h * D, axis=-1)
    return green(R, k)


def translate_fft(K: np.ndarray, Mt: np.ndarray) -> np.ndarray:
    """sum_j K[i - j] Mt[..., j] for i in [0, n)^3 by FFT (linear convolution:
    sizes 2n - 1 per axis)."""
    n = Mt.shape[-1]
    L = 2 * n - 1
    Kc = np.zeros((L, L, L), np.complex128)
    idx = np.arange(-(n - 1), n) % L
    Kc[np.ix_(idx, idx, idx)] = K
    Mp = np.zeros(Mt.shape[:-3] + (L, L, L), np.complex128)
    Mp[..., :n, :n, :n] = Mt
    out = np.fft.ifftn(np.fft.fftn(Kc)[None] * np.fft.fftn(Mp, axes=(-3, -2, -1)), axes=(-3, -2, -1))
    return out[..., :n, :n, :n]


def translate_direct(sp: BoxSplines, a: float, lo_x: np.ndarray, lo_y: np.ndarray, k: float,
                     Mt: np.ndarray) -> np.ndarray:
    """G_XY Mt with G sampled point by point (the plain form of eq:TAfactorBspline)."""
    Px, Py = grid_points(sp, a, lo_x), grid_points(sp, a, lo_y)
    Gm = green(np.linalg.norm(Px[:, None, :] - Py[None, :, :], axis=2), k)
    n = sp.n_st
    return (Mt.reshape(Mt.shape[:-3] + (n ** 3,)) @ Gm.T).reshape(Mt.shape)


def interaction_lists(leaf_idx: np.ndarray, levels: int):
    """Per level (0 = leaf): the distinct boxes (integer indices at that level),
    the box of every leaf box's ancestor, and the pairs (X, Y) translated there:
    X, Y far (Chebyshev distance of the indices > 1) and their parents near, or
    every far pair at the top level."""
    out = []
    idx = np.unique(leaf_idx, axis=0)
    anc = np.arange(len(idx))
    for l in range(levels):
        boxes, inv = np.unique(idx >> l, axis=0, return_inverse=True)
        inv = inv.ravel()
        d = np.max(np.abs(boxes[:, None, :] - boxes[None, :, :]), axis=2)
        far = d > 1
        if l + 1 < levels:
            par = boxes >> 1
            dp = np.max(np.abs(par[:, None, :] - par[None, :, :]), axis=2)
            far &= dp <= 1
        out.append(dict(boxes=boxes, leaf_to_box=inv, pairs=np.argwhere(far)))
    return idx, out


def ml_far_product(rwg: dict, k: float, x: np.ndarray, a_leaf: float, levels: int, s: int, p: int,
                   stabilise: bool = True, origin=None, fft: bool = True):
    """y = Z~_far x with the multilevel scheme (Sec. IV): equidistant-spline
    moments of the leaf boxes, moved up by the knot-insertion transfers
    (eq:interleveltransfer), transformed at every level (m~ = B^-1 C m along each
    axis), translated between the pairs of each level's interaction list
    (eq:TAfactorBspline; by FFT, or point by point), and brought down by the
    transposed maps to the test functions.  Covers exactly the pairs of leaf
    boxes that are far apart."""
    idx, lo, prot, origin = box_level(rwg, a_leaf, origin)
    sb = buffer_knots(prot, s, p)
    cfg = level_configs(s, p, sb, a_leaf, levels, k, stabilise)
    for c in cfg:
        if 2 * c.sb >= c.s - p:
            raise ValueError("buffer knots reach half a box: use larger boxes or more splines")
    leaf_boxes, lists = interaction_lists(idx, levels)
    X = np.atleast_2d(x).astype(np.complex128)
    R = X.shape[0]
    m_eq = moments(rwg, cfg[0], a_leaf, lo, transformed=False)          # (N, 4, n, n, n)
    # leaf box of every function (row of leaf_boxes)
    _, finv = np.unique(np.concatenate([leaf_boxes, idx]), axis=0, return_inverse=True)
    finv = finv.ravel()
    leaf_of = finv[len(leaf_boxes):]
    assert np.array_equal(finv[:len(leaf_boxes)], np.arange(len(leaf_boxes)))
    n0 = cfg[0].n
    M = [np.zeros((R, len(leaf_boxes), 4, n0, n0, n0), np.complex128)]
    for m in range(rwg["N"]):
        M[0][:, leaf_of[m]] += X[:, m, None, None, None, None] * m_eq[m][None]
    per_level_M = []
    Ml = M[0]
    box_of_leaf = [lists[l]["leaf_to_box"] for l in range(levels)]
    # level-0 boxes are the leaf boxes themselves (identity numbering)
    assert np.array_equal(box_of_leaf[0], np.arange(len(leaf_boxes)))
    for l in range(levels):
        if l > 0:
            child_boxes = lists[l - 1]["boxes"]
            par_of_child = np.unique(np.concatenate([lists[l]["boxes"], child_boxes >> 1]), axis=0,
                                     return_inverse=True)[1].ravel()[len(lists[l]["boxes"]):]
            Cm = transfer_matrices(cfg[l - 1], cfg[l])
            n = cfg[l].n
            Mp = np.zeros((R, len(lists[l]["boxes"]), 4, n, n, n), np.complex128)
            for cb in range(len(child_boxes)):
                c = child_boxes[cb] & 1
                Mp[:, par_of_child[cb]] += apply3(Cm[c[0]], Cm[c[1]], Cm[c[2]], per_level_M[-1][:, cb])
            Ml = Mp
        per_level_M.append(Ml)
    # translations per level (weights jk for the vector parts, 1/jk for the divergence)
    w = np.array([1j * k] * 3 + [1.0 / (1j * k)])
    Lq = []
    for l in range(levels):
        sp = cfg[l]
        a = a_leaf * 2 ** l
        boxes = lists[l]["boxes"]
        Mt = apply3(sp.A, sp.A, sp.A, per_level_M[l])                  # (R, B, 4, n', n', n')
        Zt = np.zeros_like(Mt)
        kern = {}
        for bx, by in lists[l]["pairs"]:
            off = (boxes[bx] - boxes[by]) * a
            if fft:
                key = tuple(boxes[bx] - boxes[by])
                if key not in kern:
                    kern[key] = translation_kernel(sp, a, off.astype(np.float64), k)
                Zt[:, bx] += translate_fft(kern[key], Mt[:, by])
            else:
                lo_x = origin + boxes[bx] * a
                lo_y = origin + boxes[by] * a
                Zt[:, bx] += translate_direct(sp, a, lo_x, lo_y, k, Mt[:, by])
        Zt *= w[None, None, :, None, None, None]
        Lq.append(apply3(sp.A.T, sp.A.T, sp.A.T, Zt))                 # (R, B, 4, n, n, n)
    # downward: the parents' local coefficients through the transposed transfers
    for l in range(levels - 2, -1, -1):
        child_boxes = lists[l]["boxes"]
        par_of_child = np.unique(np.concatenate([lists[l + 1]["boxes"], child_boxes >> 1]), axis=0,
                                 return_inverse=True)[1].ravel()[len(lists[l + 1]["boxes"]):]
        Cm = transfer_matrices(cfg[l], cfg[l + 1])
        for cb in range(len(child_boxes)):
            c = child_boxes[cb] & 1
            Lq[l][:, cb] += apply3(Cm[c[0]].T, Cm[c[1]].T, Cm[c[2]].T, Lq[l + 1][:, par_of_child[cb]])
    Y = np.einsum("mdijk,rmdijk->rm", m_eq, Lq[0][:, leaf_of], optimize=True)
    info = dict(configs=cfg, lists=lists, leaf_boxes=leaf_boxes, leaf_of=leaf_of, sb=sb, prot=prot, origin=origin,
                moments_eq=m_eq, level_moments=per_level_M)
    return (Y[0] if np.ndim(x) == 1 else Y), info


def leaf_far_mask(leaf_of: np.ndarray, leaf_boxes: np.ndarray) -> np.ndarray:
    """(N, N) boolean: the entries whose leaf boxes are far apart."""
    d = np.max(np.abs(leaf_boxes[:, None, :] - leaf_boxes[None, :, :]), axis=2) > 1
    return d[leaf_of][:, leaf_of]
