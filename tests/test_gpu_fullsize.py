"""Parity at the workloads' full sizes, in the launch configurations the bench
times: the 7680-unknown sphere at k = 10 and the 30720-unknown sphere at k = 20,
on sampled outputs the oracle computes one by one (matrix rows from the triangle
pairs of those rows only), and the headline solve against the oracle's full
matrix (7680 unknowns)."""
import numpy as np
import pytest
import torch

from bounds import product_bound
from oracle import cfill, efie
from oracle.mesh import flagged_pairs, rwg_table
from paper_2606_13482_amd.inputs import complex_gaussian, icosphere, planewave_set, random_directions

pytestmark = pytest.mark.gpu

_MESH = {}


def _mesh(level):
    """Mesh, RWG table and flagged triangle pairs (the near rule of the fill)."""
    if level not in _MESH:
        V, T = icosphere(level)
        rwg = rwg_table(V, T)
        _MESH[level] = (V, T, rwg, flagged_pairs(rwg, 2.0))
    return _MESH[level]


def _say(*a):
    print(*a, flush=True)


def _maxrel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.mark.parametrize("level,k,nrows,ncols", [(4, 10.0, 6, 1024), (5, 20.0, 3, 512)])
def test_full_size_sampled_rows(bie, level, k, nrows, ncols):
    """FP64 and FP32 fills, the packed FP64 product (one vector) and the split-BF16
    and FP64 block products at full size, compared on sampled rows with the
    oracle's rows.  The block products take as many columns as the bench's widest
    launches: 1024 held-out waves at 7680 unknowns, 512 grid waves at 30720."""
    V, T, rwg, flags = _mesh(level)
    N = rwg["N"]
    rng = np.random.default_rng(1000 + level)
    rows = np.unique(np.concatenate([[0, N - 1], rng.choice(N, nrows - 2, replace=False)]))
    Ro = efie.fill_rows(rwg, k, rows, flags=flags)    # (S, N)
    op = bie.Operator(V, T, k, storage="split_bf16")
    # fill: T e_i is column i = row i (T = T^T)
    E = np.zeros((rows.size, N), np.complex128)
    E[np.arange(rows.size), rows] = 1.0
    cols = op.apply(torch.from_numpy(E).cuda()).cpu().numpy()
    e_fill = _maxrel(cols, Ro)
    # packed FP64 product of one vector (the GEMV kernel)
    x = complex_gaussian(N, 7)
    y = op.apply(torch.from_numpy(x).cuda().reshape(1, -1)).cpu().numpy()[0]
    e_gemv = _maxrel(y[rows], Ro @ x)
    # block products at the bench's widest launch
    X = complex_gaussian(N, 11, cols=ncols)
    ref = X @ Ro.T                                                            # (ncols, S)
    Xd = torch.from_numpy(X).cuda()
    e_bf16 = _maxrel(op.apply(Xd, block=True).cpu().numpy()[:, rows], ref)
    e_f64 = _maxrel(op.apply(Xd, block="fp64").cpu().numpy()[:, rows], ref)
    op.close()
    op32 = bie.Operator(V, T, k, storage="c64")
    e_fill32 = _maxrel(op32.apply(torch.from_numpy(E.astype(np.complex64)).cuda()).cpu().numpy(), Ro)
    op32.close()
    _say(f"  N={N} rows {rows.tolist()}: fill FP64 {e_fill:.1e}, FP32 {e_fill32:.1e}; packed product {e_gemv:.1e}; "
         f"block products ({ncols} columns) split-BF16 {e_bf16:.1e}, FP64 {e_f64:.1e}")
    assert e_fill <= 1e-12 and e_gemv <= 1e-12 and e_f64 <= 1e-12
    assert e_fill32 <= 1e-6
    assert e_bf16 <= 3e-5


def test_full_size_headline_solve(bie):
    """The column-GMRES mixed form (split-BF16 block products, FP16 inner basis,
    FP64 refinement, continuous batch) on 16 plane waves at 7680 unknowns: every
    solution meets SCC 1e-6 against the oracle's full matrix, and the residual the
    solver reports is that SCC."""
    V, T, rwg, _ = _mesh(4)
    op = bie.Operator(V, T, 10.0, storage="split_bf16")
    d, e = planewave_set(random_directions(8, 77), "theta")
    d2, e2 = planewave_set(random_directions(8, 78), "phi")
    B = op.rhs(np.concatenate([d, d2]), np.concatenate([e, e2]))
    X, st = op.solve(B, bie.Solve(restart=50, tol=1e-6, precision="mixed", inner_tol=0.1, slots=256, basis="f16"))
    op.close()
    Zo = cfill.fill(rwg, 10.0)
    Bn, Xn = B.cpu().numpy(), X.cpu().numpy()
    res = np.linalg.norm(Bn - Xn @ Zo.T, axis=1) / np.linalg.norm(Bn, axis=1)
    rep = np.array([s["relres_true"] for s in st])
    _say(f"  headline form, 7680 unknowns: max residual {res.max():.3e}, reported {rep.max():.3e}, "
         f"iterations {int(np.mean([s['iters'] for s in st]))} mean")
    assert all(s["converged"] for s in st)
    assert res.max() <= 1e-6 * (1 + 1e-6)
    assert np.max(np.abs(rep - res) / res) <= 1e-7


def test_full_size_large_sphere_solve(bie):
    """The large-sphere form (30720 unknowns, k = 20, GMRES(30), split-BF16
    products with FP64 refinement) on 4 plane waves: converged to 1e-6, and the
    FP64 residual it is judged by agrees on sampled rows with the oracle's rows."""
    V, T, rwg, flags = _mesh(5)
    N = rwg["N"]
    op = bie.Operator(V, T, 20.0, storage="split_bf16")
    d, e = planewave_set(random_directions(4, 79), "theta")
    B = op.rhs(d, e)
    X, st = op.solve(B, bie.Solve(restart=30, tol=1e-6, precision="mixed", inner_tol=0.1, slots=256, basis="f16"))
    assert all(s["converged"] for s in st) and max(s["relres_true"] for s in st) <= 1e-6
    Rg = (B - op.apply(X)).cpu().numpy()                      # FP64 residual on the GPU
    rows = np.array([3, N // 2, N - 2])
    Ro = efie.fill_rows(rwg, 20.0, rows, flags=flags)
    Bn, Xn = B.cpu().numpy(), X.cpu().numpy()
    ro = Bn[:, rows] - Xn @ Ro.T
    scale = np.linalg.norm(Bn, axis=1)[:, None]
    err = float(np.max(np.abs(Rg[:, rows] - ro) / scale))
    _say(f"  large sphere: reported residuals {[round(s['relres_true'], 9) for s in st]}, "
         f"sampled-row residual difference {err:.1e} of |b|")
    assert err <= 1e-12
    op.close()


@pytest.mark.parametrize("terms,basis,itol", [(2, "f16", 0.01), (2, "c64", 0.1), (3, "c64", 0.1)])
def test_full_size_headline_block_solve(bie, terms, basis, itol):
    """The bench's headline form (block GMRES(50) over groups of 32 on split-BF16
    products, 2 terms, the FP16-pair inner basis and inner tolerance 1e-2 in the
    bench, FP64 refinement) on 64 plane waves at 7680 unknowns: every residual at
    most 1e-6 against the oracle's full matrix and equal to the reported SCC."""
    V, T, rwg, _ = _mesh(4)
    op = bie.Operator(V, T, 10.0, storage="split_bf16")
    d, e = planewave_set(random_directions(32, 80), "theta")
    d2, e2 = planewave_set(random_directions(32, 80), "phi")
    B = op.rhs(np.concatenate([d, d2]), np.concatenate([e, e2]))
    X, st = op.solve(B, bie.Solve(method="bgmres", block=32, restart=50, tol=1e-6, precision="mixed", inner_tol=itol,
                                  inner_terms=terms, basis=basis))
    op.close()
    Zo = cfill.fill(rwg, 10.0)
    Bn, Xn = B.cpu().numpy(), X.cpu().numpy()
    res = np.linalg.norm(Bn - Xn @ Zo.T, axis=1) / np.linalg.norm(Bn, axis=1)
    rep = np.array([s["relres_true"] for s in st])
    _say(f"  block form ({terms} terms, {basis} basis, inner {itol:g}), 7680 unknowns: max residual {res.max():.3e}, reported {rep.max():.3e}, "
         f"iterations {int(np.mean([s['iters'] for s in st]))} mean")
    assert all(s["converged"] for s in st)
    assert res.max() <= 1e-6 * (1 + 1e-6)
    assert np.max(np.abs(rep - res) / res) <= 1e-7


def test_full_size_calderon_block_solve(bie):
    """The bench's Calderon leg: Calderon-preconditioned mixed block GMRES(50)
    (groups of 32, split-BF16 products of T M with 3 terms, inner tolerance 1e-3,
    FP64 refinement) on 64 plane waves at 7680 unknowns, k = 10: every residual at most
    1e-6 against the oracle's full matrix and equal to the reported SCC; the
    preconditioner's Gram solves reach 1e-13 and M is symmetric on sampled
    entries."""
    V, T, rwg, _ = _mesh(4)
    op = bie.Operator(V, T, 10.0, storage="split_bf16")
    pc = bie.Calderon(op)
    info = pc.info()
    N = op.N
    E = torch.zeros((4, N), dtype=torch.complex128, device="cuda")
    cols = [0, 1234, 5000, N - 1]
    for a, c in enumerate(cols):
        E[a, c] = 1.0
    Mc = pc.apply(E).cpu().numpy()                      # M e_c = column c
    sym = max(abs(Mc[a, cols[b]] - Mc[b, cols[a]]) for a in range(4) for b in range(4)) / np.abs(Mc).max()
    d, e = planewave_set(random_directions(32, 81), "theta")
    d2, e2 = planewave_set(random_directions(32, 81), "phi")
    B = op.rhs(np.concatenate([d, d2]), np.concatenate([e, e2]))
    X, st = op.solve(B, bie.Solve(method="bgmres", block=32, restart=50, tol=1e-6, precision="mixed", inner_tol=1e-3,
                                  inner_terms=3, calderon=pc))
    pc.close()
    op.close()
    Zo = cfill.fill(rwg, 10.0)
    Bn, Xn = B.cpu().numpy(), X.cpu().numpy()
    res = np.linalg.norm(Bn - Xn @ Zo.T, axis=1) / np.linalg.norm(Bn, axis=1)
    rep = np.array([s["relres_true"] for s in st])
    _say(f"  Calderon block form, 7680 unknowns: max residual {res.max():.3e}, reported {rep.max():.3e}, "
         f"iterations {np.mean([s['iters'] for s in st]):.1f} mean; Gram CG {info['cg_iters']} -> "
         f"{max(info['cg_relres']):.1e}; M asymmetry {sym:.1e}")
    assert info["Nb"] == 46080 and max(info["cg_relres"]) <= 1e-13
    assert sym <= 1e-15
    assert all(s["converged"] for s in st)
    assert res.max() <= 1e-6 * (1 + 1e-6)
    assert np.max(np.abs(rep - res) / res) <= 1e-7


def test_full_size_large_sphere_block_form(bie):
    """The large sphere's timed form: block GMRES(30) over groups of 32 with 2-term
    split-BF16 products, the FP16-pair inner basis and FP64 refinement (inner tolerance 1e-2), on the first 64 waves of the 16 x 16
    (theta, phi) grid at 30720 unknowns, k = 20: every column converges, and the FP64
    residual behind the reported criterion agrees on sampled rows with the
    oracle's rows."""
    from paper_2606_13482_amd.inputs import grid_planewaves
    V, T, rwg, flags = _mesh(5)
    N = rwg["N"]
    op = bie.Operator(V, T, 20.0, storage="split_bf16")
    dirs, pols = grid_planewaves(16, 16)
    B = op.rhs(dirs[:64], pols[:64])
    X, st = op.solve(B, bie.Solve(method="bgmres", block=32, restart=30, tol=1e-6, precision="mixed",
                                  inner_tol=0.01, inner_terms=2, max_mvp=20000, basis="f16"))
    conv = [s["converged"] for s in st]
    Rg = (B - op.apply(X)).cpu().numpy()
    rows = np.array([1, N // 3, N - 1])
    Ro = efie.fill_rows(rwg, 20.0, rows, flags=flags)
    Bn, Xn = B.cpu().numpy(), X.cpu().numpy()
    ro = Bn[:, rows] - Xn @ Ro.T
    scale = np.linalg.norm(Bn, axis=1)[:, None]
    err = float(np.max(np.abs(Rg[:, rows] - ro) / scale))
    rel = np.linalg.norm(Rg, axis=1) / np.linalg.norm(Bn, axis=1)
    rep = np.array([s["relres_true"] for s in st])
    _say(f"  large sphere, block form (2 terms), 64 grid waves: converged {np.mean(conv):.3f}, max residual "
         f"{rel.max():.3e} (reported {rep.max():.3e}), iterations {np.mean([s['iters'] for s in st]):.0f} mean; "
         f"sampled-row residual difference {err:.1e} of |b|")
    assert all(conv) and rel.max() <= 1e-6 * (1 + 1e-6)
    assert np.max(np.abs(rep - rel) / rel) <= 1e-6
    assert err <= 1e-12
    op.close()


def test_pod_at_workload_size(bie):
    """POD of the learned warm-start workload's size: 256 modes from 1024 solutions
    (512 directions x theta/phi) at 7680 unknowns, k = 10.  The randomised range
    finder's singular values and projection error against the exact SVD of the same
    snapshots (the Eckart-Young optimum)."""
    from oracle import learn
    V, T, rwg, _ = _mesh(4)
    op = bie.Operator(V, T, 10.0, storage="split_bf16")
    inc = random_directions(512, 5)
    d1, e1 = planewave_set(inc, "theta")
    d2, e2 = planewave_set(inc, "phi")
    dirs, pols = np.concatenate([d1, d2]), np.concatenate([e1, e2])
    B = op.rhs(dirs, pols)
    X, st = op.solve(B, bie.Solve(method="bgmres", block=32, restart=50, tol=1e-6, precision="mixed", inner_tol=0.1,
                                  inner_terms=2, max_mvp=20000))
    assert all(s["converged"] for s in st)
    feats = bie.features(dirs, np.concatenate([np.ones(512), -np.ones(512)]))
    K = 256
    ws = bie.WarmStart.train(op, feats, X, pod_rank=K, hidden=16, epochs=0, batch=256)
    U = ws.basis().cpu().numpy()
    sg = ws.sigma()
    Xn = X.cpu().numpy()
    _, so = learn.pod(Xn, K)
    err = np.linalg.norm(Xn - (Xn @ U.conj().T) @ U)
    opt = np.sqrt(np.sum(so[K:] ** 2))
    orth = np.max(np.abs(U @ U.conj().T - np.eye(K)))
    rel = np.abs(sg - so[:K]) / so[:K]
    _say(f"  POD 256 of 1024 at 7680 unknowns: orthonormality {orth:.1e}, singular values: first 64 {rel[:64].max():.1e}, "
         f"first 128 {rel[:128].max():.1e}, all {rel.max():.1e}; projection error {err / np.linalg.norm(Xn):.4e} of "
         f"|X| (optimum {opt / np.linalg.norm(Xn):.4e}), sigma_257/sigma_1 {so[K] / so[0]:.2e}")
    # the spectrum decays slowly (sigma_257 is a quarter of sigma_1): the range
    # finder's trailing singular values are within a few per cent, the leading ones
    # exact, and the subspace it returns is within 1 % of the best rank-256 one
    assert orth <= 1e-10
    assert rel[:64].max() <= 1e-6 and rel.max() <= 3e-2
    assert err <= opt * 1.01
    ws.close()
    op.close()


def test_full_size_uneven_batch_products(bie):
    """The uneven batch at full size (64 surfaces, 648..5832 unknowns, their 1069
    plane-wave counts as columns): the grouped product of each pass in the
    batched solves' layout (16 tiles per unit; 8 columns per item on the vector
    units, 32 on the matrix cores, FP32 and FP64), on sampled rows (first, last and one random
    row of every surface) against the oracle's rows, element by element within
    the bound of each pass's arithmetic (tests/bounds.py)."""
    from paper_2606_13482_amd.inputs import uneven_batch
    probs = uneven_batch()
    ops = [bie.Operator(p["V"], p["T"], p["k"], storage="c64", keep_fp64=True) for p in probs]
    Xs = [torch.from_numpy(complex_gaussian(op.N, 500 + i, cols=len(p["dirs"])).reshape(-1, op.N)).cuda()
          for i, (op, p) in enumerate(zip(ops, probs))]
    out = {mat: [y.cpu().numpy() for y in bie.batch_apply(ops, Xs, mat=mat, unit_tiles=16, cols_per_item=cols)]
           for mat, cols in (("fp64", 8), ("fp32", 8), ("fp32_mfma", 32), ("fp64_mfma", 32))}
    worst = {mat: 0.0 for mat in out}
    rng = np.random.default_rng(77)
    for i, (op, p) in enumerate(zip(ops, probs)):
        rwg = rwg_table(p["V"], p["T"])
        N = rwg["N"]
        rows = np.unique([0, int(rng.integers(1, N - 1)), N - 1])
        Ro = efie.fill_rows(rwg, p["k"], rows, flags=flagged_pairs(rwg, 2.0))       # (S, N)
        X = Xs[i].cpu().numpy()
        ref = X @ Ro.T
        # the bound's S_i and e64 on the sampled rows: |T| restricted to them
        for mat, Y in out.items():
            b = product_bound(mat, 16, np.abs(Ro), np.abs(X))
            e = np.abs(Y[i][:, rows] - ref)
            worst[mat] = max(worst[mat], float((e / b).max()))
            assert np.all(e <= b), (i, mat, float((e / b).max()))
    _say("  uneven batch, 64 surfaces, 1069 columns: worst error / bound " +
         ", ".join(f"{m} {w:.3f}" for m, w in worst.items()))
    for op in ops:
        op.close()
