"""Pins of the oracle's solvers and convergence criteria."""
import math
import os

import numpy as np
import pytest

from oracle import cfill, efie, krylov, sampling
from paper_2606_13482_amd.inputs import complex_gaussian, planewave_set

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _c1_like(ico, level=1, k=2.0):
    rwg = ico(level)
    Z = cfill.fill(rwg, k)
    d, e = planewave_set(np.array([[0.0, 0.0, 1.0]]), "theta")
    b = efie.rhs(rwg, k, d, e)[0]
    return rwg, Z, b


def test_splitmix64_published_vector():
    want = [int(l, 16) for l in open(os.path.join(GOLDEN, "splitmix64_seed0.txt")) if l.startswith("0x")]
    g = sampling.SplitMix64(0)
    assert [g.next() for _ in range(3)] == want


def test_floyd_sample_properties():
    for n, s, seed in ((7680, 512, 1234), (480, 480, 1), (480, 479, 9), (1000, 1, 77)):
        rows = sampling.sample_rows(n, s, seed)
        assert len(rows) == min(n, s) and rows == sorted(set(rows))
        assert rows[0] >= 0 and rows[-1] < n
    # deterministic per seed, different across seeds
    assert sampling.sample_rows(7680, 512, 5) == sampling.sample_rows(7680, 512, 5)
    assert sampling.sample_rows(7680, 512, 5) != sampling.sample_rows(7680, 512, 6)


def test_floyd_uniform_marginals():
    """Every index is drawn with probability S/N (chi-square over 4000 draws)."""
    n, s, reps = 40, 10, 4000
    counts = np.zeros(n)
    for r in range(reps):
        counts[sampling.sample_rows(n, s, 1000 + r)] += 1
    expect = reps * s / n
    chi2 = np.sum((counts - expect) ** 2 / expect)
    assert chi2 < 80          # 39 dof, p ~ 1e-4


def test_full_gmres_equals_lu(ico):
    """GMRES with m >= N and a tiny tolerance is the exact Krylov solution (N = 120)."""
    rwg, Z, b = _c1_like(ico, 1)
    x_lu = krylov.lu_solve(Z, b)
    x, st = krylov.gmres(Z, b, m=rwg["N"], tol=1e-13)
    assert st.converged
    assert np.linalg.norm(x - x_lu) / np.linalg.norm(x_lu) < 1e-11
    # the Givens estimate tracks the true residual in FP64
    h = np.array(st.history)
    assert np.all(np.diff(h) <= 1e-15 * h[0])            # non-increasing within the cycle


def test_givens_estimate_matches_true_residual(ico):
    rwg, Z, b = _c1_like(ico, 2)
    for m in (5, 12):
        x, st = krylov.gmres(Z, b, m=m, tol=1e-30, max_mvp=m)
        true = np.linalg.norm(b - Z @ x) / np.linalg.norm(b)
        assert abs(st.relres_est - true) < 1e-12


def test_restarted_gmres_and_cgnr_reach_lu(ico):
    rwg, Z, b = _c1_like(ico, 2)
    x_lu = krylov.lu_solve(Z, b)
    x, st = krylov.gmres(Z, b, m=30, tol=1e-10)
    assert st.converged and st.relres_true <= 1e-10
    assert np.linalg.norm(x - x_lu) / np.linalg.norm(x_lu) < 1e-7
    x2, st2 = krylov.cgnr(Z, b, tol=1e-10, max_mvp=20000)
    assert st2.converged and st2.relres_true <= 1e-10
    assert np.linalg.norm(x2 - x_lu) / np.linalg.norm(x_lu) < 1e-7
    h = np.array(st2.history)
    # CGNR minimises ||r|| over nested spaces: non-increasing up to rounding
    assert np.all(np.diff(h) <= 1e-12)


def test_rscc_full_sample_equals_scc(ico):
    rwg, Z, b = _c1_like(ico, 2)
    x, _ = krylov.gmres(Z, b, m=30, tol=1e-3)
    n = b.shape[0]
    assert abs(krylov.rscc(Z, b, x, n, 1234) - krylov.scc(Z, b, x)) < 1e-15


def test_rscc_unbiased(ico):
    """E[eta^2] over seeds equals the squared standard residual ratio."""
    rwg, Z, b = _c1_like(ico, 2)
    x, _ = krylov.gmres(Z, b, m=30, tol=1e-2)
    s2 = krylov.scc(Z, b, x) ** 2
    vals = [krylov.rscc(Z, b, x, 48, seed) ** 2 for seed in range(3000)]
    assert abs(np.mean(vals) / s2 - 1.0) < 0.05


def test_zero_rhs_and_stops(ico):
    rwg, Z, b = _c1_like(ico, 1)
    x, st = krylov.gmres(Z, np.zeros_like(b))
    assert st.converged and st.iters == 0 and not np.any(x)
    x, st = krylov.gmres(Z, b, m=10, tol=1e-14, max_mvp=25)
    assert not st.converged and st.mvps <= 26
    x, st = krylov.cgnr(Z, np.zeros_like(b))
    assert st.converged and not np.any(x)


def test_gmres_rscc_criterion(ico):
    rwg, Z, b = _c1_like(ico, 2)
    x, st = krylov.gmres(Z, b, m=30, tol=1e-6, crit="rscc", rscc_rows=96)
    assert st.converged
    assert krylov.scc(Z, b, x) < 3e-6


def test_gmres_ccc_criterion(ico):
    """Combined criterion: with every row sampled (S = N) the RSCC equals the SCC,
    so CCC takes the SCC's iterations and solution; with a small sample the
    reported value is the SCC of the returned x and meets the tolerance."""
    rwg, Z, b = _c1_like(ico, 2)
    n = b.shape[0]
    xs, ss = krylov.gmres(Z, b, m=30, tol=1e-6, crit="scc")
    xc, sc = krylov.gmres(Z, b, m=30, tol=1e-6, crit="ccc", rscc_rows=n)
    assert sc.converged and sc.iters == ss.iters and np.allclose(xc, xs, rtol=0, atol=1e-14)
    xc, sc = krylov.gmres(Z, b, m=30, tol=1e-6, crit="ccc", rscc_rows=24, rscc_seed=5)
    assert sc.converged
    assert sc.relres_true == krylov.scc(Z, b, xc) and sc.relres_true <= 1e-6


def test_reciprocity(ico):
    """e_s . F(r; d, e_i) = e_i . F(-d; -r, e_s) since Z = Z^T (far field of Sec. II)."""
    rwg, Z, _ = _c1_like(ico, 2)
    k = 2.0
    d = np.array([0.3, -0.4, 0.866]); d /= np.linalg.norm(d)
    ei = np.cross(d, [1.0, 0, 0]); ei /= np.linalg.norm(ei)
    r = np.array([-0.6, 0.5, 0.2]); r /= np.linalg.norm(r)
    es = np.cross(r, [0, 0, 1.0]); es /= np.linalg.norm(es)
    x1 = krylov.lu_solve(Z, efie.rhs(rwg, k, d[None], ei[None])[0])
    x2 = krylov.lu_solve(Z, efie.rhs(rwg, k, -r[None], es[None])[0])
    f1 = efie.radiation_vector(rwg, k, x1, r[None])[0] @ es
    f2 = efie.radiation_vector(rwg, k, x2, -d[None])[0] @ ei
    assert abs(f1 - f2) / abs(f1) < 1e-12


def _planewaves(rwg, k, count, seed):
    from paper_2606_13482_amd.inputs import random_directions
    d, e = planewave_set(random_directions(count, seed), "theta")
    return efie.rhs(rwg, k, d, e)


def test_block_gmres_block_one_is_gmres(ico):
    """With one right-hand side per block the method is GMRES(m) itself: the same
    iteration counts and iterates as the scalar oracle (pinned to LU)."""
    rwg = ico(2)
    Z = cfill.fill(rwg, 2.0)
    B = _planewaves(rwg, 2.0, 3, 31)
    X, st = krylov.block_gmres(Z, B, m=20, tol=1e-8, block=1)
    for i in range(3):
        x, s = krylov.gmres(Z, B[i], m=20, tol=1e-8)
        assert st[i].converged and s.converged
        assert st[i].iters == s.iters
        assert np.linalg.norm(X[i] - x) / np.linalg.norm(x) < 1e-10


def test_block_gmres_minimal_residual_brute_force(ico):
    """One cycle of j block steps gives, for every column, the minimiser of
    ||b_i - Z x|| over the block Krylov space span{B, ZB, ..., Z^{j-1} B}: checked
    against least squares over that space built explicitly (N = 120, 4 columns,
    j = 3).  A dropped Hessenberg block, a wrong least-squares right side or a
    wrong scaling moves the result off the minimiser."""
    rwg = ico(1)
    Z = cfill.fill(rwg, 2.0)
    B = _planewaves(rwg, 2.0, 4, 32)
    j = 3
    X, st = krylov.block_gmres(Z, B, m=j, tol=1e-30, block=4, max_mvp=j)
    K = [B.T]
    for _ in range(j - 1):
        K.append(Z @ K[-1])
    K, _ = np.linalg.qr(np.concatenate(K, axis=1))                 # N x jq
    ZK = Z @ K
    for i in range(4):
        c = np.linalg.lstsq(ZK, B[i], rcond=None)[0]
        xb = K @ c
        assert np.linalg.norm(X[i] - xb) / np.linalg.norm(xb) < 1e-9
        # the cycle's estimate is the true residual of the minimiser
        rt = np.linalg.norm(B[i] - Z @ X[i]) / np.linalg.norm(B[i])
        assert abs(st[i].relres_est - rt) <= 1e-9 * rt
        assert abs(st[i].relres_true - rt) <= 1e-12 * rt
    # and a larger block space never does worse than each column's own space
    for i in range(4):
        xs, _ = krylov.gmres(Z, B[i], m=j, tol=1e-30, max_mvp=j)
        assert np.linalg.norm(B[i] - Z @ X[i]) <= np.linalg.norm(B[i] - Z @ xs) * (1 + 1e-12)


def test_block_gmres_full_space_equals_lu(ico):
    """When the block Krylov space reaches the whole space (j q >= N) the method
    solves exactly: equals LU (N = 120, 4 columns)."""
    rwg = ico(1)
    Z = cfill.fill(rwg, 2.0)
    B = _planewaves(rwg, 2.0, 4, 33)
    X, st = krylov.block_gmres(Z, B, m=40, tol=1e-12, block=4)
    Xl = np.linalg.solve(Z, B.T).T
    assert all(s.converged for s in st)
    assert np.max(np.linalg.norm(X - Xl, axis=1) / np.linalg.norm(Xl, axis=1)) < 1e-9
    assert max(s.iters for s in st) <= 30


def test_block_gmres_dependent_columns(ico):
    """Dependent right-hand sides (a repeat and a sum) are deflated from the
    initial block: the block keeps 2 directions and every solution is still the
    linear image of the independent ones."""
    rwg = ico(2)
    Z = cfill.fill(rwg, 2.0)
    b = _planewaves(rwg, 2.0, 2, 34)
    B = np.stack([b[0], b[1], b[0], 2.0 * b[0] - 1j * b[1]])
    X, st = krylov.block_gmres(Z, B, m=30, tol=1e-9, block=4)
    assert all(s.converged for s in st)
    Xl = np.linalg.solve(Z, B.T).T
    assert np.max(np.linalg.norm(X - Xl, axis=1) / np.linalg.norm(Xl, axis=1)) < 1e-6
    assert np.linalg.norm(X[2] - X[0]) <= 1e-8 * np.linalg.norm(X[0])


def test_block_gmres_breakdown_on_invariant_space():
    """A matrix with three distinct eigenvalues: the block Krylov space of two
    right-hand sides stops growing after three steps (partial breakdown), and the
    solution is then exact."""
    rng = np.random.default_rng(3)
    N = 60
    Q, _ = np.linalg.qr(rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N)))
    lam = np.repeat([1.0, 2.0 + 1.0j, -0.5 + 0.3j], N // 3)
    Z = (Q * lam) @ np.linalg.inv(Q)
    B = rng.standard_normal((2, N)) + 1j * rng.standard_normal((2, N))
    X, st = krylov.block_gmres(Z, B, m=30, tol=1e-11, block=2)
    assert all(s.converged for s in st)
    assert max(s.iters for s in st) <= 3
    assert np.max(np.linalg.norm(B - X @ Z.T, axis=1) / np.linalg.norm(B, axis=1)) < 1e-11


def test_block_gmres_restarts_and_zero_rhs(ico):
    """Restarted block GMRES reaches the standard criterion for every column,
    with fewer block steps per right-hand side than GMRES(m) per column; a zero
    right-hand side gives x = 0 at once."""
    rwg = ico(2)
    Z = cfill.fill(rwg, 2.0)
    B = _planewaves(rwg, 2.0, 8, 35)
    B[3] = 0.0
    X, st = krylov.block_gmres(Z, B, m=10, tol=1e-8, block=4)
    res = np.linalg.norm(B - X @ Z.T, axis=1)
    nb = np.linalg.norm(B, axis=1)
    assert all(s.converged for s in st)
    assert np.all(res <= 1e-8 * nb * (1 + 1e-9))
    assert st[3].iters == 0 and np.all(X[3] == 0)
    its = [krylov.gmres(Z, B[i], m=10, tol=1e-8)[1].iters for i in range(8) if i != 3]
    assert np.mean([st[i].iters for i in range(8) if i != 3]) < np.mean(its)
