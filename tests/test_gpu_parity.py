"""GPU path against the FP64 oracle, through the C ABI (libbie.so).

Tolerances: FP64 matrix and products 1e-10 (max-norm and Frobenius relative),
FP32 matrix entries 1e-5 relative to max|T|, solutions to the 1e-6 criterion.
"""
import math
import sys

import numpy as np
import pytest
import torch

from oracle import cfill, efie, krylov
from oracle.mesh import flagged_pairs, rwg_table
from paper_2606_13482_amd.inputs import complex_gaussian, cube_sphere, icosphere, planewave_set

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


CASES = {}


def case(level, k):
    key = (level, k)
    if key not in CASES:
        V, T = icosphere(level)
        rwg = rwg_table(V, T)
        CASES[key] = (V, T, rwg, cfill.fill(rwg, k))
    return CASES[key]


def rel_err(A, B):
    return (np.max(np.abs(A - B)) / np.max(np.abs(B)), np.linalg.norm(A - B) / np.linalg.norm(B))


@pytest.mark.parametrize("level,k", [(1, 2.0), (2, 2.0), (3, 6.0)])
def test_fill_fp64(bie, level, k):
    _say(f"fill fp64 level={level} k={k}")
    V, T, rwg, Zo = case(level, k)
    op = bie.Operator(V, T, k)
    assert op.N == rwg["N"]
    assert np.array_equal(op.edges()[:, :2], rwg["edges"])
    assert np.array_equal(op.edges()[:, 2], rwg["tp"]) and np.array_equal(op.edges()[:, 3], rwg["tm"])
    Z = op.matrix().cpu().numpy()
    emax, efro = rel_err(Z, Zo)
    _say("  max/fro rel err", emax, efro)
    assert emax <= 1e-10 and efro <= 1e-10
    assert np.array_equal(Z, Z.T)                      # bitwise symmetric


def test_near_pairs_equal_oracle(bie):
    V, T, rwg, _ = case(3, 6.0)
    op = bie.Operator(V, T, 6.0)
    got = {tuple(p) for p in op.near_pairs()}
    fl = flagged_pairs(rwg)
    want = {(int(p), int(q)) for p, q in zip(*np.nonzero(np.triu(fl)))}
    assert got == want


@pytest.mark.parametrize("level,k", [(2, 2.0), (3, 6.0)])
def test_fill_fp32(bie, level, k):
    _say(f"fill fp32 level={level} k={k}")
    V, T, rwg, Zo = case(level, k)
    op = bie.Operator(V, T, k, storage="c64")
    Z = op.matrix(torch.complex64).cpu().numpy().astype(np.complex128)
    emax, efro = rel_err(Z, Zo)
    _say("  max/fro rel err", emax, efro)
    assert emax <= 1e-5 and efro <= 1e-5
    assert np.array_equal(Z, Z.T)


def test_rhs_and_farfield(bie):
    V, T, rwg, Zo = case(2, 2.0)
    k = 2.0
    op = bie.Operator(V, T, k)
    inc = np.array([[0.2, -0.3, 0.93], [0.0, 0.0, 1.0], [1.0, 0.0, 0.0]])
    d, e = planewave_set(inc, "theta")
    B = op.rhs(d, e).cpu().numpy()
    Bo = efie.rhs(rwg, k, d, e)
    assert np.max(np.abs(B - Bo)) / np.max(np.abs(Bo)) < 1e-12
    x = complex_gaussian(op.N, 11, cols=2)
    obs = np.array([[0, 0, 1.0], [0.6, 0.0, 0.8], [-1.0, 0, 0]])
    F = op.farfield(torch.from_numpy(x).cuda(), obs).cpu().numpy()
    for r in range(2):
        Fo = efie.radiation_vector(rwg, k, x[r], obs)
        assert np.max(np.abs(F[r] - Fo)) / np.max(np.abs(Fo)) < 1e-12
    # bistatic RCS (bie_rcs) against the oracle's, and non-unit directions refused
    S = op.rcs(torch.from_numpy(x).cuda(), obs).cpu().numpy()
    for r in range(2):
        So = efie.rcs(rwg, k, x[r], obs)
        assert np.max(np.abs(S[r] - So)) / np.max(So) < 1e-12
    with pytest.raises(bie.BieError):
        op.rcs(torch.from_numpy(x).cuda(), 2.0 * obs)


@pytest.mark.parametrize("R", [1, 3, 6])
def test_apply_fp64_and_conj(bie, R):
    V, T, rwg, Zo = case(3, 6.0)
    op = bie.Operator(V, T, 6.0)
    x = complex_gaussian(op.N, 7, cols=R)
    X = torch.from_numpy(x).cuda()
    Y = op.apply(X).cpu().numpy()
    Yc = op.apply(X, conj=True).cpu().numpy()
    for r in range(R):
        yo = Zo @ x[r]
        assert np.linalg.norm(Y[r] - yo) / np.linalg.norm(yo) < 1e-10
        yc = Zo.conj().T @ x[r]
        assert np.linalg.norm(Yc[r] - yc) / np.linalg.norm(yc) < 1e-10


def test_apply_fp32(bie):
    V, T, rwg, Zo = case(3, 6.0)
    op = bie.Operator(V, T, 6.0, storage="c64")
    x = complex_gaussian(op.N, 7, cols=2)
    Y = op.apply(torch.from_numpy(x.astype(np.complex64)).cuda()).cpu().numpy()
    for r in range(2):
        yo = Zo @ x[r]
        assert np.linalg.norm(Y[r] - yo) / np.linalg.norm(yo) < 1e-5


def test_gmres_c1_plain_fp64(bie):
    """480 unknowns, k = 2, GMRES(30), SCC 1e-6 (the small sphere workload)."""
    _say("gmres c1")
    V, T, rwg, Zo = case(2, 2.0)
    op = bie.Operator(V, T, 2.0)
    d, e = planewave_set(np.array([[0.0, 0.0, 1.0]]), "theta")
    B = op.rhs(d, e)
    X, st = op.solve(B, bie.Solve(restart=30, tol=1e-6))
    x = X.cpu().numpy()[0]
    b = B.cpu().numpy()[0]
    _say("  stats", st[0])
    assert st[0]["converged"]
    res = np.linalg.norm(b - Zo @ x) / np.linalg.norm(b)
    assert res <= 1e-6 * (1 + 1e-9)
    x_or, st_or = krylov.gmres(Zo, b, m=30, tol=1e-6)
    assert abs(st[0]["iters"] - st_or.iters) <= 2
    x_lu = krylov.lu_solve(Zo, b)
    fwd = np.linalg.norm(x - x_lu) / np.linalg.norm(x_lu)
    fwd_or = np.linalg.norm(x_or - x_lu) / np.linalg.norm(x_lu)
    _say("  forward error gpu/oracle", fwd, fwd_or)
    assert fwd < 3 * fwd_or + 1e-9
    # tight solve reaches the direct solution
    X2, st2 = op.solve(B, bie.Solve(restart=30, tol=1e-11))
    assert np.linalg.norm(X2.cpu().numpy()[0] - x_lu) / np.linalg.norm(x_lu) < 1e-8


def test_cgnr_c1(bie):
    V, T, rwg, Zo = case(2, 2.0)
    op = bie.Operator(V, T, 2.0)
    d, e = planewave_set(np.array([[0.0, 0.0, 1.0]]), "theta")
    B = op.rhs(d, e)
    X, st = op.solve(B, bie.Solve(method="cgnr", tol=1e-6, max_mvp=20000))
    x = X.cpu().numpy()[0]
    b = B.cpu().numpy()[0]
    _say("  cgnr stats", st[0])
    assert st[0]["converged"]
    assert np.linalg.norm(b - Zo @ x) / np.linalg.norm(b) <= 1e-6 * (1 + 1e-9)
    x_or, st_or = krylov.cgnr(Zo, b, tol=1e-6, max_mvp=20000)
    assert abs(st[0]["iters"] - st_or.iters) <= max(3, st_or.iters // 50)


def test_rscc_criterion(bie):
    V, T, rwg, Zo = case(2, 2.0)
    op = bie.Operator(V, T, 2.0)
    d, e = planewave_set(np.array([[0.3, 0.1, 0.9]]), "phi")
    B = op.rhs(d, e)
    X, st = op.solve(B, bie.Solve(restart=30, tol=1e-6, crit="rscc", rscc_rows=96, rscc_seed=77))
    assert st[0]["converged"]
    x = X.cpu().numpy()[0]; b = B.cpu().numpy()[0]
    # the criterion value reported is the oracle's RSCC for the same x and the same row sample
    want = krylov.rscc(Zo, b, x, 96, 77 + st[0]["checks"] - 1)
    assert abs(st[0]["relres_true"] - want) <= 1e-9 * want
    assert krylov.scc(Zo, b, x) < 5e-6


def test_ccc_criterion(bie):
    """Combined criterion (RSCC gates, SCC confirms): converged columns report the
    SCC of their solution against the oracle matrix; with every row sampled it
    takes the SCC's iterations."""
    V, T, rwg, Zo = case(2, 2.0)
    op = bie.Operator(V, T, 2.0)
    d, e = planewave_set(np.array([[0.3, 0.1, 0.9], [0.0, 0.0, 1.0], [1.0, 0.2, -0.3]]), "phi")
    B = op.rhs(d, e)
    X, st = op.solve(B, bie.Solve(restart=30, tol=1e-6, crit="ccc", rscc_rows=48, rscc_seed=3))
    Xn, Bn = X.cpu().numpy(), B.cpu().numpy()
    for r in range(B.shape[0]):
        want = krylov.scc(Zo, Bn[r], Xn[r])
        assert st[r]["converged"] and abs(st[r]["relres_true"] - want) <= 1e-9 * want and want <= 1e-6
    Xs, sts = op.solve(B, bie.Solve(restart=30, tol=1e-6))
    Xa, sta = op.solve(B, bie.Solve(restart=30, tol=1e-6, crit="ccc", rscc_rows=op.N))
    assert [s["iters"] for s in sta] == [s["iters"] for s in sts]
    assert torch.equal(Xa, Xs)
    with pytest.raises(bie.BieError):
        op.solve(B[:1], bie.Solve(crit="ccc", precision="mixed"))


@pytest.mark.parametrize("nrhs", [5, 20])
def test_multi_rhs_equals_single(bie, nrhs):
    """Columns solved together equal their single solves bitwise."""
    V, T, rwg, Zo = case(2, 2.0)
    op = bie.Operator(V, T, 2.0)
    inc = np.array([[0, 0, 1.0], [0.3, 0.1, 0.9], [1.0, 0, 0], [0, -1.0, 0], [0.5, 0.5, 0.5]])
    if nrhs > len(inc):
        from paper_2606_13482_amd.inputs import random_directions
        inc = np.concatenate([inc, random_directions(nrhs - len(inc), 12)])
    d, e = planewave_set(inc, "theta")
    B = op.rhs(d, e)
    X, st = op.solve(B, bie.Solve(restart=30, tol=1e-8))
    for r in range(B.shape[0]):
        Xs, sts = op.solve(B[r:r + 1].clone(), bie.Solve(restart=30, tol=1e-8))
        assert sts[0]["iters"] == st[r]["iters"]
        assert torch.equal(Xs[0], X[r])


def test_edge_cases(bie):
    V, T, rwg, Zo = case(2, 2.0)
    op = bie.Operator(V, T, 2.0)
    B = torch.zeros((2, op.N), dtype=torch.complex128, device="cuda")
    d, e = planewave_set(np.array([[0, 0, 1.0]]), "theta")
    B[1] = op.rhs(d, e)[0]
    X, st = op.solve(B, bie.Solve(tol=1e-6))
    assert st[0]["converged"] and st[0]["iters"] == 0 and torch.count_nonzero(X[0]) == 0
    assert st[1]["converged"]
    # warm start at the solution: no iterations
    X2, st2 = op.solve(B[1:2], bie.Solve(tol=1e-6), x0=X[1:2])
    assert st2[0]["converged"] and st2[0]["iters"] == 0
    # cap -> not converged, best iterate returned
    X3, st3 = op.solve(B[1:2], bie.Solve(tol=1e-14, max_mvp=12, restart=10))
    assert not st3[0]["converged"] and st3[0]["mvps"] <= 13
    # NaN -> ENUMERIC
    Bn = B[1:2].clone(); Bn[0, 3] = float("nan")
    with pytest.raises(bie.BieError) as ei:
        op.solve(Bn)
    assert ei.value.code == bie.BIE_ENUMERIC


def test_determinism(bie):
    V, T, rwg, _ = case(3, 6.0)
    a = bie.Operator(V, T, 6.0).matrix()
    b = bie.Operator(V, T, 6.0).matrix()
    assert torch.equal(a, b)


def test_cube_sphere_family(bie):
    """Ellipsoid and rounded cube (uneven-batch families) against the oracle."""
    for fam in ("ellipsoid", "rounded_cube"):
        V, T = cube_sphere(6, fam, axes=(1.0, 1.7, 2.4))
        rwg = rwg_table(V, T)
        k = 3.0
        Zo = cfill.fill(rwg, k)
        op = bie.Operator(V, T, k)
        emax, efro = rel_err(op.matrix().cpu().numpy(), Zo)
        assert emax <= 1e-10 and efro <= 1e-10


def test_fp32_matrix_solve(bie):
    """FP32-stored matrix, FP64 vectors and accumulation: converged on the FP32
    matrix; the FP64 residual is limited by the FP32 rounding of the entries."""
    V, T, rwg, Zo = case(2, 2.0)
    op = bie.Operator(V, T, 2.0, storage="c64")
    d, e = planewave_set(np.array([[0.0, 0.0, 1.0]]), "theta")
    B = op.rhs(d, e)
    X, st = op.solve(B, bie.Solve(restart=30, tol=1e-6))
    assert st[0]["converged"]
    x = X.cpu().numpy()[0]; b = B.cpu().numpy()[0]
    assert np.linalg.norm(b - Zo @ x) / np.linalg.norm(b) < 2e-6


@pytest.mark.parametrize("level,k,inner", [(2, 2.0, 1e-3), (3, 6.0, 1e-3), (3, 6.0, 1e-6)])
def test_mixed_precision_refinement(bie, level, k, inner):
    """FP32 inner GMRES + FP64 iterative refinement reaches the FP64 criterion;
    the residual is checked with the oracle matrix and the solution against LU."""
    V, T, rwg, Zo = case(level, k)
    op = bie.Operator(V, T, k, storage="c64", keep_fp64=True)
    inc = np.array([[0.0, 0.0, 1.0], [0.4, -0.2, 0.9]])
    d, e = planewave_set(inc, "theta")
    B = op.rhs(d, e)
    X, st = op.solve(B, bie.Solve(restart=30, tol=1e-6, precision="mixed", inner_tol=inner))
    Bn = B.cpu().numpy(); Xn = X.cpu().numpy()
    for r in range(2):
        assert st[r]["converged"], st[r]
        res = np.linalg.norm(Bn[r] - Zo @ Xn[r]) / np.linalg.norm(Bn[r])
        assert res <= 1e-6 * (1 + 1e-6), res
        assert abs(res - st[r]["relres_true"]) <= 1e-9
        x_lu = krylov.lu_solve(Zo, Bn[r])
        xp, stp = krylov.gmres(Zo, Bn[r], m=30, tol=1e-6)
        fwd = np.linalg.norm(Xn[r] - x_lu) / np.linalg.norm(x_lu)
        fwd_p = np.linalg.norm(xp - x_lu) / np.linalg.norm(x_lu)
        assert fwd < 10 * fwd_p + 1e-9
    # the FP32 matrix is the rounding of the FP64 one
    Z32 = op.matrix(torch.complex64).cpu().numpy()
    assert np.array_equal(Z32, Zo.astype(np.complex64)) or np.max(np.abs(Z32 - Zo)) / np.max(np.abs(Zo)) < 1e-7


@pytest.mark.parametrize("R", [1, 3, 130, 300])
def test_block_product_split_bf16(bie, R):
    """Split-BF16 block product on MFMA (FP32 accumulation) against the FP64 oracle:
    about 16 significant bits per entry, so 2e-5 relative to ||T x||."""
    V, T, rwg, Zo = case(3, 6.0)
    op = bie.Operator(V, T, 6.0, storage="split_bf16")
    x = complex_gaussian(op.N, 21, cols=R)
    Y = op.apply(torch.from_numpy(x).cuda(), block=True).cpu().numpy()
    Yo = x @ Zo.T
    err = np.linalg.norm(Y - Yo, axis=1) / np.linalg.norm(Yo, axis=1)
    _say(f"  block product R={R}: max rel err {err.max():.2e}")
    assert err.max() < 2e-5
    # the FP64 product of the same operator is unaffected
    Y64 = op.apply(torch.from_numpy(x[:1]).cuda()).cpu().numpy()
    assert np.linalg.norm(Y64[0] - Yo[0]) / np.linalg.norm(Yo[0]) < 1e-10


@pytest.mark.parametrize("R", [1, 3, 65, 130])
def test_block_product_fp64(bie, R):
    """FP64 block product on the matrix cores (dense FP64 copy, v_mfma_f64_16x16x4f64)
    against the oracle matrix: FP64 rounding only, so 1e-13 relative to ||T x||;
    and against the packed FP64 product of the same operator."""
    V, T, rwg, Zo = case(3, 6.0)
    op = bie.Operator(V, T, 6.0)
    x = complex_gaussian(op.N, 23, cols=R)
    X = torch.from_numpy(x).cuda()
    Y = op.apply(X, block="fp64").cpu().numpy()
    Yo = x @ Zo.T
    err = np.linalg.norm(Y - Yo, axis=1) / np.linalg.norm(Yo, axis=1)
    Yp = op.apply(X).cpu().numpy()
    errp = np.linalg.norm(Y - Yp, axis=1) / np.linalg.norm(Yp, axis=1)
    _say(f"  FP64 block product R={R}: max rel err {err.max():.2e} (vs packed {errp.max():.2e})")
    assert err.max() < 1e-13 and errp.max() < 1e-13


@pytest.mark.parametrize("terms", [3, 2])
def test_mixed_refinement_split_bf16_block(bie, terms):
    """Block GMRES (simultaneous columns) on the split-BF16 matrix with FP64 refinement
    (inner products with 3 terms, or 2: BF16-rounded vectors)."""
    V, T, rwg, Zo = case(3, 6.0)
    op = bie.Operator(V, T, 6.0, storage="split_bf16")
    from paper_2606_13482_amd.inputs import random_directions
    inc = random_directions(24, 3)
    d, e = planewave_set(inc, "theta")
    B = op.rhs(d, e)
    itol = 1e-3 if terms == 3 else 1e-1
    X, st = op.solve(B, bie.Solve(restart=30, tol=1e-6, precision="mixed", inner_tol=itol, inner_terms=terms))
    Bn = B.cpu().numpy(); Xn = X.cpu().numpy()
    res = np.linalg.norm(Bn - Xn @ Zo.T, axis=1) / np.linalg.norm(Bn, axis=1)
    _say(f"  block mixed ({terms} terms): max residual", res.max(), "outer checks", max(s["checks"] for s in st),
         "iterations", sum(s["iters"] for s in st))
    assert all(s["converged"] for s in st)
    assert res.max() <= 1e-6 * (1 + 1e-6)


def test_fp16_basis_refinement(bie):
    """FP16 storage of the inner Krylov basis (split-BF16 products, FP64
    refinement): converged to 1e-6 against the oracle matrix, with about the
    iterations of the complex64 basis; the option is refused where it does not
    apply."""
    V, T, rwg, Zo = case(3, 6.0)
    op = bie.Operator(V, T, 6.0, storage="split_bf16")
    from paper_2606_13482_amd.inputs import random_directions
    inc = random_directions(16, 21)
    d, e = planewave_set(inc, "theta")
    B = op.rhs(d, e)
    Bn = B.cpu().numpy()
    out = {}
    for basis in ("c64", "f16"):
        X, st = op.solve(B, bie.Solve(restart=30, tol=1e-6, precision="mixed", inner_tol=0.1, basis=basis))
        res = np.linalg.norm(Bn - X.cpu().numpy() @ Zo.T, axis=1) / np.linalg.norm(Bn, axis=1)
        assert all(s["converged"] for s in st), basis
        assert res.max() <= 1e-6 * (1 + 1e-6), (basis, res.max())
        out[basis] = sum(s["iters"] for s in st)
        _say(f"  {basis} basis: max residual {res.max():.2e}, iterations {out[basis]}")
    assert out["f16"] <= 1.25 * out["c64"]
    with pytest.raises(bie.BieError):
        op.solve(B[:1], bie.Solve(basis="f16"))   # plain precision
    op64 = bie.Operator(V, T, 6.0, storage="c64", keep_fp64=True)
    with pytest.raises(bie.BieError):
        op64.solve(B[:1], bie.Solve(precision="mixed", basis="f16"))   # FP32 storage


@pytest.mark.parametrize("storage,basis", [("split_bf16", "c64"), ("c64", "c64"), ("split_bf16", "f16")])
def test_continuous_batch_bitwise(bie, storage, basis):
    """The refinement engine keeps a fixed number of right-hand sides in flight and
    hands the slot of a converged one to the next.  Every column is computed on its
    own (block product columns, Arnoldi, FP64 residual), so each solution is bitwise
    the same whatever the number of slots, including one right-hand side alone
    (complex64 or FP16 inner Krylov basis)."""
    V, T, rwg, Zo = case(3, 6.0)
    op = bie.Operator(V, T, 6.0, storage=storage, keep_fp64=(storage == "c64"))
    from paper_2606_13482_amd.inputs import random_directions
    inc = random_directions(19, 8)
    d, e = planewave_set(inc, "phi")
    B = op.rhs(d, e)
    base = bie.Solve(restart=20, tol=1e-6, precision="mixed", inner_tol=1e-2, basis=basis)
    X0, st0 = op.solve(B, base)
    for slots in (3, 4, 17, 64):
        Xs, sts = op.solve(B, bie.Solve(**{**base.__dict__, "slots": slots}))
        assert torch.equal(Xs, X0), slots
        assert [s["iters"] for s in sts] == [s["iters"] for s in st0]
    X1, st1 = op.solve(B[5:6], base)
    assert torch.equal(X1[0], X0[5])
    Bn = B.cpu().numpy(); Xn = X0.cpu().numpy()
    res = np.linalg.norm(Bn - Xn @ Zo.T, axis=1) / np.linalg.norm(Bn, axis=1)
    _say(f"  {storage} ({basis} basis): max residual {res.max():.2e}, iterations {[s['iters'] for s in st0]}")
    assert all(s["converged"] for s in st0)
    assert res.max() <= 1e-6 * (1 + 1e-6)
    for r in range(len(st0)):
        assert abs(res[r] - st0[r]["relres_true"]) <= 1e-9


def test_continuous_batch_warm_and_zero_rhs(bie):
    """Initial guesses of mixed quality (exact, perturbed, zero) and a zero right-hand
    side in one continuous batch with fewer slots than right-hand sides."""
    V, T, rwg, Zo = case(3, 6.0)
    op = bie.Operator(V, T, 6.0, storage="split_bf16")
    from paper_2606_13482_amd.inputs import random_directions
    inc = random_directions(6, 9)
    d, e = planewave_set(inc, "theta")
    B = op.rhs(d, e)
    B[2] = 0
    Bn = B.cpu().numpy()
    xs = np.array([krylov.lu_solve(Zo, b) if np.any(b) else np.zeros_like(b) for b in Bn])
    x0 = xs.copy()
    x0[1] *= 1.0 + 1e-3
    x0[3] = 0
    x0[4] = complex_gaussian(op.N, 4)
    X, st = op.solve(B, bie.Solve(restart=20, tol=1e-6, precision="mixed", inner_tol=1e-2, slots=2),
                     x0=torch.from_numpy(x0).cuda())
    Xn = X.cpu().numpy()
    assert all(s["converged"] for s in st)
    assert np.all(Xn[2] == 0) and st[2]["iters"] == 0
    assert st[0]["iters"] == 0 and st[0]["checks"] == 1       # exact guess: one FP64 check
    res = np.linalg.norm(Bn - Xn @ Zo.T, axis=1) / np.maximum(np.linalg.norm(Bn, axis=1), 1e-300)
    res[2] = 0.0
    assert res.max() <= 1e-6 * (1 + 1e-6)
    assert st[1]["iters"] < st[3]["iters"]                     # a near guess saves iterations


@pytest.mark.parametrize("mixed", [False, True])
def test_initial_guess_fallback(bie, mixed):
    """use_x0 = 2: a guess no better than zero (||b - T x0|| >= ||b||) is replaced by
    zero from the solver's first residual; a good guess is kept.  The dropped guess
    gives the same iterations as a solve from zero."""
    V, T, rwg, Zo = case(3, 6.0)
    op = bie.Operator(V, T, 6.0, storage="split_bf16" if mixed else "c128")
    from paper_2606_13482_amd.inputs import random_directions
    d, e = planewave_set(random_directions(3, 21), "theta")
    B = op.rhs(d, e)
    Bn = B.cpu().numpy()
    x0 = np.array([krylov.lu_solve(Zo, b) for b in Bn]) * (1.0 + 1e-4)
    x0[1] = 30.0 * complex_gaussian(op.N, 5)      # far worse than zero
    opts = bie.Solve(restart=20, tol=1e-6, precision="mixed" if mixed else "plain", inner_tol=1e-2)
    X, st = op.solve(B, opts, x0=torch.from_numpy(x0).cuda(), x0_fallback=True)
    Xz, stz = op.solve(B[1:2], opts)
    assert [s["x0_kept"] for s in st] == [1, 0, 1]
    assert all(s["converged"] for s in st)
    assert st[1]["iters"] == stz[0]["iters"]
    assert st[0]["iters"] < stz[0]["iters"] and st[2]["iters"] < stz[0]["iters"]
    res = np.linalg.norm(Bn - X.cpu().numpy() @ Zo.T, axis=1) / np.linalg.norm(Bn, axis=1)
    assert res.max() <= 1e-6 * (1 + 1e-6)
