"""The 7680-unknown sphere (icosphere level 4, radius 1 m, k = 10) with one
x-polarised plane wave from +z, solved on the GPU in plain FP64 and with the
FP32 fill (mixed precision, FP64 refinement), against the oracle: residual on
the oracle's full matrix, forward error against the oracle's LU solution (with
a condition estimate), and the bistatic RCS from bie_rcs against the oracle's
RCS and the Mie series, the threshold frozen from the oracle's own deviation
(tests/golden/sphere7680_rcs_oracle.txt, written by make_sphere7680_rcs.py)."""
import math
import os

import numpy as np
import pytest
import scipy.linalg as sla
import torch

from oracle import cfill
from oracle.mesh import rwg_table
from paper_2606_13482_amd.inputs import icosphere, planewave_set

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "sphere7680_rcs_oracle.txt")


def _say(*a):
    print(*a, flush=True)


def _golden():
    kv, rows = {}, []
    for line in open(GOLDEN):
        if line.startswith("#"):
            continue
        if "=" in line:
            k, v = line.split("=")
            kv[k.strip()] = float(v)
        else:
            rows.append([float(t) for t in line.split()])
    return kv, np.array(rows)


@pytest.fixture(scope="module")
def c2():
    """Mesh, the oracle's matrix, LU solution and condition estimate."""
    V, T = icosphere(4)
    rwg = rwg_table(V, T)
    Zo = cfill.fill(rwg, 10.0)
    d, e = planewave_set(np.array([[0.0, 0.0, 1.0]]), "theta")
    from oracle import efie
    b = efie.rhs(rwg, 10.0, d, e)[0]
    lu, piv = sla.lu_factor(Zo)
    xo = sla.lu_solve((lu, piv), b)
    rcond, _ = sla.lapack.zgecon(lu, np.linalg.norm(Zo, 1), norm="1")
    del lu
    return dict(V=V, T=T, rwg=rwg, Z=Zo, b=b, xo=xo, kappa=1.0 / rcond, d=d, e=e)


def _check(Zo, b, xo, x):
    res = np.linalg.norm(b - Zo @ x) / np.linalg.norm(b)
    fwd = np.linalg.norm(x - xo) / np.linalg.norm(xo)
    return res, fwd


def _cuts(theta_deg):
    th = np.radians(theta_deg)
    return (np.stack([np.sin(th), 0 * th, np.cos(th)], 1), np.stack([0 * th, np.sin(th), np.cos(th)], 1))


def test_plain_fp64_against_lu_and_mie(bie, c2):
    kv, g = _golden()
    op = bie.Operator(c2["V"], c2["T"], 10.0)
    assert op.N == 7680 == int(kv["N"])
    B = op.rhs(c2["d"], c2["e"])
    assert np.max(np.abs(B.cpu().numpy()[0] - c2["b"])) <= 1e-12 * np.max(np.abs(c2["b"]))
    out = {}
    for tol in (1e-6, 1e-10):
        X, st = op.solve(B, bie.Solve(restart=50, tol=tol, max_mvp=40000))
        res, fwd = _check(c2["Z"], c2["b"], c2["xo"], X.cpu().numpy()[0])
        out[tol] = (res, fwd, st[0]["iters"], X)
        assert st[0]["converged"] and res <= tol * (1 + 1e-6)
    _say(f"  kappa_1 estimate {c2['kappa']:.3e} (golden {kv['kappa1_estimate']:.3e}); plain FP64 GMRES(50): "
         + "; ".join(f"tol {t:g}: residual {r:.2e}, forward error {f:.2e}, {i} iterations"
                     for t, (r, f, i, _) in out.items()))
    assert abs(c2["kappa"] / kv["kappa1_estimate"] - 1) < 0.05
    # the forward error at residual r is bounded by the condition number times r
    for r, f, _, _ in out.values():
        assert f <= c2["kappa"] * r
    # tightened to 1e-10 the solution is within 1e-6 of the oracle's LU solution
    assert out[1e-10][1] <= 1e-6
    # bistatic RCS on the E- and H-plane cuts (bie_rcs)
    e_plane, h_plane = _cuts(g[:, 0])
    X = out[1e-6][3]
    s_e = op.rcs(X, e_plane).cpu().numpy()[0]
    s_h = op.rcs(X, h_plane).cpu().numpy()[0]
    gpu = np.concatenate([s_e, s_h])
    mie_ref = np.concatenate([g[:, 1], g[:, 2]])
    orc = np.concatenate([g[:, 3], g[:, 4]])
    d_oracle = float(np.sqrt(np.mean((gpu - orc) ** 2) / np.mean(orc ** 2)))
    d_mie = float(np.sqrt(np.mean((gpu - mie_ref) ** 2) / np.mean(mie_ref ** 2)))
    _say(f"  RCS: rms deviation from the oracle's {d_oracle:.2e}, from Mie {d_mie:.4f} "
         f"(oracle's own {kv['rms_rel_error_oracle_vs_mie']:.4f})")
    assert d_oracle <= 1e-4
    assert d_mie <= kv["rms_rel_error_oracle_vs_mie"] + 1e-3
    # backscatter (theta = 179 deg on both cuts is next to it): Mie gives 0.929 pi a^2 at ka = 10
    op.close()


def test_fp32_fill_mixed_solve(bie, c2):
    """FP32 fill and storage (regular pairs in FP32, touching and near pairs in
    FP64) with the FP64 copy for refinement: inner GMRES(50) on the FP32 matrix,
    FP64 residuals and criterion; the solution meets 1e-6 on the oracle's matrix."""
    op = bie.Operator(c2["V"], c2["T"], 10.0, storage="c64", keep_fp64=True)
    B = op.rhs(c2["d"], c2["e"])
    X, st = op.solve(B, bie.Solve(restart=50, tol=1e-6, precision="mixed", inner_tol=1e-3, max_mvp=40000))
    res, fwd = _check(c2["Z"], c2["b"], c2["xo"], X.cpu().numpy()[0])
    _say(f"  FP32 fill, mixed precision: residual {res:.2e} (reported {st[0]['relres_true']:.2e}), "
         f"forward error {fwd:.2e}, {st[0]['iters']} iterations, {st[0]['checks']} FP64 checks")
    assert st[0]["converged"] and res <= 1e-6 * (1 + 1e-6)
    assert abs(st[0]["relres_true"] - res) <= 1e-7 * res
    assert fwd <= c2["kappa"] * res
    op.close()
