"""Dense Galerkin EFIE matrix, plane-wave right-hand side and far field (oracle).

Operator (Sec. II, eq:efie, eq:discretizedEFIE):  T = jk T_A - (jk)^-1 T_Phi with
    [T_A]_mn   =  int int f_m(x) . g(x,y) f_n(y)
    [T_Phi]_mn = -int int div f_m(x) g(x,y) div f_n(y)          (eq:matTA, eq:matTPhi)
    g(x,y) = exp(-jk|x-y|) / (4 pi |x-y|),   time convention exp(+j w t).
RWG functions without edge-length normalisation (Sec. II): on triangle p of
f_m, f_m = s_p (r - v_p)/(2 A_p) and div f_m = s_p / A_p (s_p = +1 on c+,
-1 on c-, v_p the free vertex).  Hence

    Z_mn = sum_{p in m} sum_{q in n} s_p s_q / (A_p A_q)
           [ (jk/4) int_p int_q (x - v_p).(y - v_q) g  +  (1/(jk)) int_p int_q g ]

(the two minus signs of T_Phi cancel).  With a rule of area-relative weights w
on both triangles the areas cancel:
    Z_mn += s_p s_q sum_ij w_i w_j [ (jk/4)(x_i - v_p).(y_j - v_q) + 1/(jk) ] g(|x_i - y_j|).

Flagged pairs (touching or near, see mesh.flagged_pairs) use singularity
subtraction g = g_r + 1/(4 pi R), g_r = (exp(-jkR) - 1)/(4 pi R) (limit -jk/(4 pi)
at R = 0) on the same product rule, plus the static part with the inner
integral in closed form (potentials.k0_k1) at the outer points; the value is
the mean of the two orderings (p outer / q inner and q outer / p inner).
These singular-pair choices are readings: the paper does not discuss them.

Right-hand side (Sec. II):  [e]_m = int f_m . e_inc,  e_inc = pol exp(-jk d.r).
Far field (Sec. II, radiation potentials): for the unknown j (current
normalised by the wave impedance, Sec. II) the scattered far field is
    E_s ~ -jk exp(-jkr)/(4 pi r) (I - rr) . F,   F(r) = int j(y) exp(jk r.y) dS,
so the bistatic RCS for a unit-amplitude plane wave is (k^2/(4 pi)) |r x F|^2.
"""
from __future__ import annotations

import math

import numpy as np

from .mesh import flagged_pairs, triangle_edges
from .potentials import k0_k1
from .quadrature import points, radon7

FOUR_PI = 4.0 * math.pi


def green(R: np.ndarray, k: float) -> np.ndarray:
    """g(R) = exp(-jkR)/(4 pi R)."""
    return np.exp(-1j * k * R) / (FOUR_PI * R)


def green_regular(R: np.ndarray, k: float) -> np.ndarray:
    """g_r(R) = (exp(-jkR) - 1)/(4 pi R), evaluated as (-2 sin^2(kR/2) - j sin kR)/(4 pi R),
    with the limit -jk/(4 pi) at R = 0."""
    R = np.asarray(R, dtype=np.float64)
    safe = np.where(R > 0, R, 1.0)
    s = np.sin(0.5 * k * safe)
    val = (-2.0 * s * s - 1j * np.sin(k * safe)) / (FOUR_PI * safe)
    return np.where(R > 0, val, -1j * k / FOUR_PI)


class Geometry:
    """Per-triangle data the fill needs: quadrature points, free vertices, RWG slots."""

    def __init__(self, rwg: dict, rule=None):
        self.rwg = rwg
        self.bary, self.w = rule if rule is not None else radon7()
        V, T = rwg["V"], rwg["T"]
        self.X = points(V, T, self.bary)             # (F, nq, 3)
        self.Vf = V[T]                               # (F, 3, 3): free vertex of slot a is T[t,a]
        self.m_of, self.s_of = triangle_edges(rwg)   # (F,3)
        self.tri = V[T]                              # vertex coordinates (F,3,3), CCW


def _regular_blocks(G: Geometry, pidx: np.ndarray, qidx: np.ndarray, k: float):
    """J (P,Q,3,3) = sum_ij w_i w_j g (x_i - v_a).(y_j - v_b) and J0 (P,Q) = sum_ij w_i w_j g."""
    Xp = G.X[pidx]; Xq = G.X[qidx]
    R = np.linalg.norm(Xp[:, None, :, None, :] - Xq[None, :, None, :, :], axis=-1)  # (P,Q,i,j)
    W = G.w[:, None] * G.w[None, :]
    Gm = W[None, None] * green(R, k)
    Dp = Xp[:, None, :, :] - G.Vf[pidx][:, :, None, :]      # (P,3a,i,3)
    Dq = Xq[:, None, :, :] - G.Vf[qidx][:, :, None, :]      # (Q,3b,j,3)
    M = np.einsum("pqij,qbjc->pqibc", Gm, Dq, optimize=True)
    J = np.einsum("paic,pqibc->pqab", Dp, M, optimize=True)
    J0 = Gm.sum(axis=(2, 3))
    return J, J0


def singular_block(G: Geometry, p: int, q: int, k: float, orderings: bool = False):
    """Singularity-subtracted J (3,3) and J0 for one flagged pair (mean of both orderings).

    orderings: also return the static parts of the two orderings separately,
    ((Jsp, J0sp), (Jsq, J0sq)) with p outer / q inner and q outer / p inner; they
    are equal in exact integration, so their difference measures the outer rule's
    error on the pair."""
    rwg = G.rwg
    w = G.w
    Xp, Xq = G.X[p], G.X[q]
    vp, vq = G.Vf[p], G.Vf[q]                  # (3,3) free vertices per slot
    Ap, Aq = rwg["area"][p], rwg["area"][q]
    R = np.linalg.norm(Xp[:, None, :] - Xq[None, :, :], axis=-1)
    Gr = (w[:, None] * w[None, :]) * green_regular(R, k)
    Dp = Xp[None, :, :] - vp[:, None, :]       # (a,i,3)
    Dq = Xq[None, :, :] - vq[:, None, :]       # (b,j,3)
    J = np.einsum("ij,aic,bjc->ab", Gr, Dp, Dq)
    J0 = Gr.sum()
    # p outer, closed-form inner integral over q
    K0q, K1q = k0_k1(Xp, G.tri[q])
    # int_q (y - v_b)/R = K1 + (x - v_b) K0
    Iq = K1q[None, :, :] + (Xp[None, :, :] - vq[:, None, :]) * K0q[None, :, None]   # (b,i,3)
    Jsp = np.einsum("i,aic,bic->ab", w, Dp, Iq) / (FOUR_PI * Aq)
    J0sp = np.dot(w, K0q) / (FOUR_PI * Aq)
    # q outer, closed-form inner integral over p
    K0p, K1p = k0_k1(Xq, G.tri[p])
    Ip = K1p[None, :, :] + (Xq[None, :, :] - vp[:, None, :]) * K0p[None, :, None]   # (a,j,3)
    Jsq = np.einsum("j,bjc,ajc->ab", w, Dq, Ip) / (FOUR_PI * Ap)
    J0sq = np.dot(w, K0p) / (FOUR_PI * Ap)
    if orderings:
        return J + 0.5 * (Jsp + Jsq), J0 + 0.5 * (J0sp + J0sq), ((Jsp, J0sp), (Jsq, J0sq))
    return J + 0.5 * (Jsp + Jsq), J0 + 0.5 * (J0sp + J0sq)


def local_blocks(G: Geometry, pidx: np.ndarray, k: float, near_factor: float = 2.0,
                 flags: np.ndarray | None = None, singular: bool = True):
    """Local 3x3 blocks LB (P,F,3,3) = s_a s_b [(jk/4) J + J0/(jk)] and the
    vector / scalar parts separately (for structural checks)."""
    F = G.rwg["F"]
    qidx = np.arange(F)
    J, J0 = _regular_blocks(G, pidx, qidx, k)
    if singular:
        if flags is None:
            flags = flagged_pairs(G.rwg, near_factor)
        for ip, p in enumerate(pidx):
            for q in np.nonzero(flags[p])[0]:
                J[ip, q], J0[ip, q] = singular_block(G, int(p), int(q), k)
    S = G.s_of[pidx][:, None, :, None] * G.s_of[None, :, None, :]
    jk = 1j * k
    LA = S * (0.25 * J)                      # contributes with factor jk
    LP = S * J0[:, :, None, None]            # contributes with factor 1/(jk)
    return LA, LP, jk


def fill(rwg: dict, k: float, rule=None, near_factor: float = 2.0, singular: bool = True,
         parts: bool = False, chunk: int = 16):
    """Full N x N complex128 matrix Z (and, if parts, A and P with Z = jk A + P/(jk),
    A = T_A and P = -T_Phi)."""
    G = Geometry(rwg, rule)
    N, F = rwg["N"], rwg["F"]
    flags = flagged_pairs(rwg, near_factor) if singular else None
    A = np.zeros(N * N, np.complex128)
    P = np.zeros(N * N, np.complex128)
    for p0 in range(0, F, chunk):
        pidx = np.arange(p0, min(F, p0 + chunk))
        LA, LP, jk = local_blocks(G, pidx, k, near_factor, flags, singular)
        rows = G.m_of[pidx][:, None, :, None]
        cols = G.m_of[None, :, None, :]
        idx = (rows * N + cols).reshape(-1)
        for tgt, src in ((A, LA), (P, LP)):
            v = src.reshape(-1)
            tgt += np.bincount(idx, weights=v.real, minlength=N * N) \
                + 1j * np.bincount(idx, weights=v.imag, minlength=N * N)
    A = A.reshape(N, N); P = P.reshape(N, N)
    jk = 1j * k
    Z = jk * A + P / jk
    return (Z, A, P) if parts else Z


def fill_rows(rwg: dict, k: float, rows, rule=None, near_factor: float = 2.0, flags=None):
    """Rows Z[rows, :] computed from the triangle pairs of those rows only
    (flags: the flagged-pair matrix of mesh.flagged_pairs, if already at hand)."""
    rows = np.asarray(rows, dtype=np.int64)
    G = Geometry(rwg, rule)
    N = rwg["N"]
    if flags is None:
        flags = flagged_pairs(rwg, near_factor)
    tris = np.unique(np.concatenate([rwg["tp"][rows], rwg["tm"][rows]]))
    out = np.zeros((rows.size, N), np.complex128)
    for c0 in range(0, tris.size, 16):
        pidx = tris[c0:c0 + 16]
        LA, LP, jk = local_blocks(G, pidx, k, near_factor, flags, True)
        L = jk * LA + LP / jk                                     # (P,F,3,3)
        for ip, p in enumerate(pidx):
            for a in range(3):
                m = G.m_of[p, a]
                hit = np.nonzero(rows == m)[0]
                if hit.size == 0:
                    continue
                cols = G.m_of.reshape(-1)                        # (F*3,) over (q,b)
                v = L[ip, :, a, :].reshape(-1)
                row = np.bincount(cols, weights=v.real, minlength=N) \
                    + 1j * np.bincount(cols, weights=v.imag, minlength=N)
                out[hit] += row
    return out


def rhs(rwg: dict, k: float, dirs: np.ndarray, pols: np.ndarray, rule=None) -> np.ndarray:
    """B (R,N): [e]_m = sum_{p in m} (s_p/2) sum_i w_i (x_i - v_p).pol exp(-jk d.x_i)."""
    G = Geometry(rwg, rule)
    dirs = np.atleast_2d(dirs); pols = np.atleast_2d(pols)
    N, F = rwg["N"], rwg["F"]
    B = np.zeros((dirs.shape[0], N), np.complex128)
    for r in range(dirs.shape[0]):
        ph = np.exp(-1j * k * (G.X @ dirs[r]))                       # (F,i)
        D = G.X[:, None, :, :] - G.Vf[:, :, None, :]                   # (F,a,i,3)
        val = 0.5 * G.s_of * np.einsum("i,fai,fi->fa", G.w, D @ pols[r], ph)
        idx = G.m_of.reshape(-1)
        v = val.reshape(-1)
        B[r] = np.bincount(idx, weights=v.real, minlength=N) + 1j * np.bincount(idx, weights=v.imag, minlength=N)
    return B


def radiation_vector(rwg: dict, k: float, x: np.ndarray, obs: np.ndarray, rule=None) -> np.ndarray:
    """F(r) = int j(y) exp(jk r.y) dS for the coefficient vector x (N,), directions obs (M,3)."""
    G = Geometry(rwg, rule)
    obs = np.atleast_2d(obs)
    ph = np.exp(1j * k * np.einsum("fic,mc->mfi", G.X, obs))          # (M,F,i)
    D = G.X[:, None, :, :] - G.Vf[:, :, None, :]                        # (F,a,i,3)
    coef = 0.5 * G.s_of * x[G.m_of]                                    # (F,a)
    return np.einsum("fa,i,faic,mfi->mc", coef, G.w, D, ph)


def rcs(rwg: dict, k: float, x: np.ndarray, obs: np.ndarray, rule=None) -> np.ndarray:
    """Bistatic RCS (m^2) for a unit-amplitude incident wave: (k^2/4pi) |r x F|^2."""
    obs = np.atleast_2d(obs)
    Fv = radiation_vector(rwg, k, x, obs, rule)
    tang = Fv - np.sum(obs * Fv, axis=1, keepdims=True) * obs
    return k * k / FOUR_PI * np.sum(np.abs(tang) ** 2, axis=1)


def scalar_single_layer(rwg: dict, k: float, rule=None, near_factor: float = 2.0) -> np.ndarray:
    """V (F,F), V_pq = (1/(A_p A_q)) int_p int_q g, with the same quadrature and
    singular treatment as the fill (piecewise-constant single layer of Sec. VI-A)."""
    G = Geometry(rwg, rule)
    F = rwg["F"]
    flags = flagged_pairs(rwg, near_factor)
    Vm = np.zeros((F, F), np.complex128)
    for p0 in range(0, F, 16):
        pidx = np.arange(p0, min(F, p0 + 16))
        _, J0 = _regular_blocks(G, pidx, np.arange(F), k)
        for ip, p in enumerate(pidx):
            for q in np.nonzero(flags[p])[0]:
                J0[ip, q] = singular_block(G, int(p), int(q), k)[1]
        Vm[pidx] = J0
    return Vm
