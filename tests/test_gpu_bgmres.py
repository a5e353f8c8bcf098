"""Block GMRES on the GPU (method "bgmres") against the oracle's block GMRES, LU
and the GPU's own column GMRES."""
import numpy as np
import pytest
import torch

from oracle import cfill, krylov
from oracle.mesh import rwg_table
from paper_2606_13482_amd.inputs import complex_gaussian, icosphere, planewave_set, random_directions

pytestmark = pytest.mark.gpu

_CACHE = {}


def _case(level, k):
    key = (level, k)
    if key not in _CACHE:
        V, T = icosphere(level)
        rwg = rwg_table(V, T)
        _CACHE[key] = (V, T, rwg, cfill.fill(rwg, k))
    return _CACHE[key]


def _say(*a):
    print(*a, flush=True)


def _rhs(op, count, seed):
    d, e = planewave_set(random_directions(count, seed), "theta")
    return op.rhs(d, e)


def _res(Zo, B, X):
    Bn, Xn = B.cpu().numpy(), X.cpu().numpy()
    return np.linalg.norm(Bn - Xn @ Zo.T, axis=1) / np.linalg.norm(Bn, axis=1)


@pytest.mark.parametrize("block,m", [(4, 10), (3, 7), (8, 20)])
def test_bgmres_fp64_matches_oracle(bie, block, m):
    """Plain FP64 block GMRES: the iterations of the oracle's block GMRES on the
    same right-hand sides (ragged last block when block does not divide R), every
    residual within tol against the oracle matrix, solutions equal to the
    oracle's within the tolerance's reach."""
    V, T, rwg, Zo = _case(2, 2.0)
    op = bie.Operator(V, T, 2.0)
    B = _rhs(op, 10, 40)
    X, st = op.solve(B, bie.Solve(method="bgmres", block=block, restart=m, tol=1e-8))
    Xo, so = krylov.block_gmres(Zo, B.cpu().numpy(), m=m, tol=1e-8, block=block)
    res = _res(Zo, B, X)
    it, ito = [s["iters"] for s in st], [s.iters for s in so]
    fwd = np.linalg.norm(X.cpu().numpy() - Xo, axis=1) / np.linalg.norm(Xo, axis=1)
    _say(f"  block {block} m {m}: iterations GPU {it} oracle {ito}; max residual {res.max():.2e}; vs oracle {fwd.max():.1e}")
    assert all(s["converged"] for s in st)
    assert res.max() <= 1e-8 * (1 + 1e-6)
    assert it == ito
    assert fwd.max() <= 1e-6
    rep = np.array([s["relres_true"] for s in st])
    assert np.max(np.abs(rep - res) / res) <= 1e-6


def test_bgmres_block_one_is_gmres(bie):
    """Block size 1: the GPU's column GMRES iterations and solutions."""
    V, T, rwg, Zo = _case(2, 2.0)
    op = bie.Operator(V, T, 2.0)
    B = _rhs(op, 5, 41)
    X1, s1 = op.solve(B, bie.Solve(method="bgmres", block=1, restart=20, tol=1e-8))
    X0, s0 = op.solve(B, bie.Solve(method="gmres", restart=20, tol=1e-8))
    d = (torch.linalg.vector_norm(X1 - X0, dim=1) / torch.linalg.vector_norm(X0, dim=1)).max().item()
    _say(f"  block 1 iterations {[s['iters'] for s in s1]} column GMRES {[s['iters'] for s in s0]}; difference {d:.1e}")
    assert [s["iters"] for s in s1] == [s["iters"] for s in s0]
    assert d <= 1e-9


def test_bgmres_full_space_and_dependent_columns(bie):
    """On 120 unknowns a block of 4 fills the space within 30 steps: the solutions
    equal LU.  Repeated and combined right-hand sides are deflated from the
    starting block and still solved."""
    V, T, rwg, Zo = _case(1, 2.0)
    op = bie.Operator(V, T, 2.0)
    B = _rhs(op, 4, 42)
    X, st = op.solve(B, bie.Solve(method="bgmres", block=4, restart=40, tol=1e-12))
    Xl = np.linalg.solve(Zo, B.cpu().numpy().T).T
    e = np.max(np.linalg.norm(X.cpu().numpy() - Xl, axis=1) / np.linalg.norm(Xl, axis=1))
    Bd = torch.stack([B[0], B[1], B[0], 2.0 * B[0] - 1j * B[1]])
    Xd, sd = op.solve(Bd, bie.Solve(method="bgmres", block=4, restart=30, tol=1e-9))
    rd = _res(Zo, Bd, Xd)
    dup = (torch.linalg.vector_norm(Xd[2] - Xd[0]) / torch.linalg.vector_norm(Xd[0])).item()
    _say(f"  full space vs LU {e:.1e} in {max(s['iters'] for s in st)} steps; dependent columns residual {rd.max():.1e}, "
         f"repeat {dup:.1e}")
    assert all(s["converged"] for s in st) and e <= 1e-9 and max(s["iters"] for s in st) <= 30
    assert all(s["converged"] for s in sd) and rd.max() <= 1e-9 * (1 + 1e-6) and dup <= 1e-8


def test_bgmres_zero_rhs_and_initial_guess(bie):
    """A zero right-hand side gives x = 0; a given initial guess is kept and
    counted; fallback (use_x0 = 2) replaces a guess worse than zero."""
    V, T, rwg, Zo = _case(2, 2.0)
    op = bie.Operator(V, T, 2.0)
    B = _rhs(op, 4, 43)
    B[2] = 0.0
    X, st = op.solve(B, bie.Solve(method="bgmres", block=4, restart=20, tol=1e-8))
    assert st[2]["converged"] and st[2]["iters"] == 0 and torch.all(X[2] == 0)
    res = _res(Zo, B[[0, 1, 3]], X[[0, 1, 3]])
    assert res.max() <= 1e-8 * (1 + 1e-6)
    x0 = torch.from_numpy(30.0 * complex_gaussian(op.N, 5, cols=4)).cuda()
    x0[0] = X[0] * (1 + 1e-3)
    X2, s2 = op.solve(B, bie.Solve(method="bgmres", block=4, restart=20, tol=1e-8), x0=x0, x0_fallback=True)
    _say(f"  x0 kept {[s['x0_kept'] for s in s2]}, iterations {[s['iters'] for s in s2]}")
    assert s2[0]["x0_kept"] == 1 and s2[1]["x0_kept"] == 0
    assert all(s["converged"] for s in s2)
    assert _res(Zo, B[[0, 1, 3]], X2[[0, 1, 3]]).max() <= 1e-8 * (1 + 1e-6)
    assert s2[0]["iters"] < st[0]["iters"]


@pytest.mark.parametrize("basis", ["c64", "f16"])
def test_bgmres_mixed_precision(bie, basis):
    """Mixed precision (split-BF16 products, complex64 or FP16-pair inner basis,
    FP64 refinement) on 1920 unknowns at k = 6 with 32 plane waves: every
    residual at most 1e-6 against the oracle matrix, in fewer products per
    right-hand side than the column GMRES of the same mixed form; the FP16 basis
    within a fifth more products than the complex64 one."""
    V, T, rwg, Zo = _case(3, 6.0)
    op = bie.Operator(V, T, 6.0, storage="split_bf16")
    B = _rhs(op, 32, 44)
    X, st = op.solve(B, bie.Solve(method="bgmres", block=16, restart=30, tol=1e-6, precision="mixed",
                                  inner_tol=0.1, basis=basis))
    Xc, sc = op.solve(B, bie.Solve(restart=30, tol=1e-6, precision="mixed", inner_tol=0.1))
    res = _res(Zo, B, X)
    mb, mc = np.mean([s["mvps"] for s in st]), np.mean([s["mvps"] for s in sc])
    _say(f"  mixed, {basis} basis: block max residual {res.max():.2e}, products per RHS {mb:.0f} (column GMRES {mc:.0f})")
    assert all(s["converged"] for s in st)
    assert res.max() <= 1e-6 * (1 + 1e-6)
    assert mb < mc
    if basis == "f16":
        _, s64 = op.solve(B, bie.Solve(method="bgmres", block=16, restart=30, tol=1e-6, precision="mixed",
                                       inner_tol=0.1))
        assert mb <= 1.2 * np.mean([s["mvps"] for s in s64])


def test_bgmres_rejections(bie):
    V, T, rwg, Zo = _case(1, 2.0)
    op = bie.Operator(V, T, 2.0)
    B = _rhs(op, 2, 45)
    for opts in (bie.Solve(method="bgmres", block=33), bie.Solve(method="bgmres", crit="rscc"),
                 bie.Solve(method="bgmres", precision="mixed")):
        with pytest.raises(bie.BieError):
            op.solve(B, opts)
    ops = bie.Operator(V, T, 2.0, star=True)
    with pytest.raises(bie.BieError):
        ops.solve(B, bie.Solve(method="bgmres"))


def test_bgmres_slots_and_cap(bie):
    """slots > 0 solves the right-hand sides in consecutive chunks (each chunk
    grouped on its own; every residual still within tol against the oracle
    matrix); max_mvp caps the products and the call reports not converged."""
    V, T, rwg, Zo = _case(2, 2.0)
    op = bie.Operator(V, T, 2.0)
    B = _rhs(op, 10, 46)
    X, st = op.solve(B, bie.Solve(method="bgmres", block=4, restart=10, tol=1e-8, slots=4))
    res = _res(Zo, B, X)
    _say(f"  chunks of 4: iterations {[s['iters'] for s in st]}, max residual {res.max():.2e}")
    assert all(s["converged"] for s in st) and res.max() <= 1e-8 * (1 + 1e-6)
    Xc, sc = op.solve(B, bie.Solve(method="bgmres", block=4, restart=10, tol=1e-14, max_mvp=25))
    _say(f"  cap 25: products {[s['mvps'] for s in sc]}, converged {[s['converged'] for s in sc]}")
    assert not any(s["converged"] for s in sc)
    assert all(s["mvps"] <= 25 + 10 for s in sc)
    rc = _res(Zo, B, Xc)
    assert np.all(rc < 1.0) and np.all(np.abs(np.array([s["relres_true"] for s in sc]) - rc) <= 1e-6 * rc)
