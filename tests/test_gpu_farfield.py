"""The single-level B-spline far field on the GPU (bie_far_*) against the
oracle (oracle/bspline.py): the same cubes (integer-equal), the same buffer,
the far product to FP64 rounding, and both within the interpolation error of
the dense oracle's far entries."""
import numpy as np
import pytest
import torch

from oracle import bspline as bs
from oracle import cfill, efie
from oracle.mesh import flagged_pairs, rwg_table
from paper_2606_13482_amd.inputs import complex_gaussian, icosphere

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("p,s", [(3, 8), (1, 6), (5, 10)])
def test_far_product_matches_oracle(bie, p, s):
    V, T = icosphere(3)
    rwg = rwg_table(V, T)
    k, a = 2.0, 0.7
    op = bie.Operator(V, T, k)
    far = bie.FarField(op, a, s, p)
    info = far.info()
    idx, lo, prot, origin = bs.box_level(rwg, a)
    assert np.array_equal(far.boxes(), idx)
    assert abs(info["protrusion"] - prot) <= 1e-12 and info["buffer_knots"] == bs.buffer_knots(prot, s, p)
    X = complex_gaussian(op.N, 21, cols=3)
    Y = far.apply(torch.from_numpy(X).cuda()).cpu().numpy()
    Yo, oi = bs.far_product(rwg, k, X, a, s, p)
    err = np.linalg.norm(Y - Yo) / np.linalg.norm(Yo)
    Y1 = far.apply(torch.from_numpy(X[1:2].copy()).cuda()).cpu().numpy()[0]
    msg = f"  p={p} s={s}: {info['boxes']} cubes, {info['far_pairs']} far pairs, buffer {info['buffer_knots']}, " \
          f"{info['points_per_axis']} points per axis; GPU vs oracle {err:.2e}"
    if p == 3:
        Z = cfill.fill(rwg, k)
        F = bs.far_mask(oi["inv"], oi["far"])
        Yd = X @ (Z * F).T
        e_dense = np.linalg.norm(Y - Yd) / np.linalg.norm(Yd)
        msg += f", vs dense far entries {e_dense:.2e}"
        assert e_dense <= 1e-3
    _say(msg)
    assert err <= 1e-12
    assert np.array_equal(Y1, Y[1])          # columns are independent
    far.close()
    op.close()


def test_far_product_workload_sphere(bie):
    """The 7680-unknown sphere at k = 10 with cubes of 0.4 m (s = 8, p = 3): the GPU
    far product on two sampled target cubes against the oracle's interpolated
    blocks, and on sampled rows against the dense oracle's far entries."""
    V, T = icosphere(4)
    rwg = rwg_table(V, T)
    k, a, s, p = 10.0, 0.4, 8, 3
    op = bie.Operator(V, T, k)
    far = bie.FarField(op, a, s, p)
    info = far.info()
    x = complex_gaussian(op.N, 22)
    y = far.apply(torch.from_numpy(x).cuda().reshape(1, -1)).cpu().numpy()[0]
    idx, lo, prot, origin = bs.box_level(rwg, a)
    assert np.array_equal(far.boxes(), idx)
    sb = bs.buffer_knots(prot, s, p)
    sp = bs.BoxSplines(s, p, sb)
    boxes, inv, farm = bs.far_pairs(idx)
    members = [np.nonzero(inv == b)[0] for b in range(len(boxes))]
    rng = np.random.default_rng(5)
    targets = rng.choice(len(boxes), 2, replace=False)
    mt = bs.moments(rwg, sp, a, lo)
    box_lo = origin + boxes * a
    err_o, err_d = [], []
    flags = flagged_pairs(rwg, 2.0)
    for t in targets:
        rows = members[t]
        yo = np.zeros(rows.size, np.complex128)
        for b in np.nonzero(farm[t])[0]:
            yo += bs.far_block(mt, rows, members[b], sp, a, box_lo[t], box_lo[b], k) @ x[members[b]]
        err_o.append(np.linalg.norm(y[rows] - yo) / np.linalg.norm(yo))
        sample = rows[:3]
        Zr = efie.fill_rows(rwg, k, sample, flags=flags)
        fcols = np.isin(inv, np.nonzero(farm[t])[0])
        yd = Zr[:, fcols] @ x[fcols]
        err_d.append(np.linalg.norm(y[sample] - yd) / np.linalg.norm(yd))
    _say(f"  7680 unknowns, k = 10, cubes 0.4 m: {info['boxes']} cubes, {info['far_pairs']} far pairs, buffer "
         f"{info['buffer_knots']}; GPU vs oracle {max(err_o):.2e}, vs dense far entries {max(err_d):.2e}")
    assert max(err_o) <= 1e-12
    assert max(err_d) <= 5e-3
    far.close()
    op.close()


def test_far_rejections(bie):
    V, T = icosphere(2)
    op = bie.Operator(V, T, 2.0)
    for box, s, p in ((0.7, 8, 2), (0.7, 3, 3), (-1.0, 8, 3), (0.4, 6, 3)):
        with pytest.raises(bie.BieError):
            bie.FarField(op, box, s, p)
    op.close()


# ----------------------------------------------------------------------------- multilevel (bie_farml_*)
@pytest.mark.parametrize("k,pairs", [(2.0, [5256, 386]), (6.0, [5256, 386])])
def test_multilevel_matches_oracle(bie, k, pairs):
    """Two levels (cubes of 0.35 m and 0.7 m) on the 1920-unknown sphere, cubic
    splines, s = 8: k = 2 keeps s on the parent level (Sec. IV-C), k = 6 doubles
    it to 2 s - p (Sec. IV-D); the GPU product (knot-insertion transfers, FFT
    translations of sizes 16 and 32) against the oracle's multilevel product to
    FP64 rounding, the level data equal, and within the interpolation error of
    the dense oracle's entries between far leaf cubes."""
    V, T = icosphere(3)
    rwg = rwg_table(V, T)
    a, s, p = 0.35, 8, 3
    op = bie.Operator(V, T, k)
    far = bie.FarFieldML(op, a, 2, s, p)
    X = complex_gaussian(op.N, 31, cols=2)
    Y = far.apply(torch.from_numpy(X).cuda()).cpu().numpy()
    Yo, oi = bs.ml_far_product(rwg, k, X, a, 2, s, p)
    err = np.linalg.norm(Y - Yo) / np.linalg.norm(Yo)
    infos = [far.level_info(l) for l in range(2)]
    for l, (inf, cfg, L) in enumerate(zip(infos, oi["configs"], oi["lists"])):
        assert inf["boxes"] == len(L["boxes"]) and inf["far_pairs"] == len(L["pairs"]) == pairs[l]
        assert inf["buffer_knots"] == cfg.sb and inf["splines"] == cfg.n and inf["points_per_axis"] == cfg.n_st
    Z = cfill.fill(rwg, k)
    F = bs.leaf_far_mask(oi["leaf_of"], oi["leaf_boxes"])
    Yd = X @ (Z * F).T
    e_dense = np.linalg.norm(Y - Yd) / np.linalg.norm(Yd)
    _say(f"  k={k:g}: levels {[(i['boxes'], i['far_pairs'], i['splines'], i['points_per_axis']) for i in infos]}; "
         f"GPU vs oracle {err:.2e}, vs dense far entries {e_dense:.2e}")
    assert err <= 1e-12
    assert e_dense <= 2e-3
    far.close()
    op.close()


def test_multilevel_one_level_is_single_level(bie):
    """One level: the multilevel product (FFT translations) equals the
    single-level far field (lattice-table translations) to FP64 rounding."""
    V, T = icosphere(3)
    k, a, s, p = 2.0, 0.7, 8, 3
    op = bie.Operator(V, T, k)
    f1 = bie.FarField(op, a, s, p)
    fm = bie.FarFieldML(op, a, 1, s, p)
    x = torch.from_numpy(complex_gaussian(op.N, 32, cols=1)).cuda()
    y1, ym = f1.apply(x).cpu().numpy(), fm.apply(x).cpu().numpy()
    assert np.linalg.norm(y1 - ym) <= 1e-12 * np.linalg.norm(y1)
    assert fm.level_info(0)["far_pairs"] == f1.info()["far_pairs"]
    f1.close()
    fm.close()
    op.close()


def test_multilevel_three_levels_against_dense(bie):
    """Three levels (cubes of 0.2, 0.4 and 0.8 m) on the 7680-unknown sphere at
    k = 2: the far product against the operator's own dense FP64 matrix masked
    to the far leaf cubes (cubes from the oracle's box rule), within 2e-3; every
    level translates pairs, the pairs of all levels cover the far leaf pairs."""
    V, T = icosphere(4)
    rwg = rwg_table(V, T)
    k, a, s, p = 2.0, 0.2, 8, 3
    op = bie.Operator(V, T, k)
    far = bie.FarFieldML(op, a, 3, s, p)
    infos = [far.level_info(l) for l in range(3)]
    assert all(i["far_pairs"] > 0 for i in infos)
    idx, lo, prot, origin = bs.box_level(rwg, a)
    leaf_boxes, lists = bs.interaction_lists(idx, 3)
    assert [len(L["pairs"]) for L in lists] == [i["far_pairs"] for i in infos]
    _, finv = np.unique(np.concatenate([leaf_boxes, idx]), axis=0, return_inverse=True)
    leaf_of = finv.ravel()[len(leaf_boxes):]
    F = torch.from_numpy(bs.leaf_far_mask(leaf_of, leaf_boxes)).cuda()
    Z = op.matrix()
    X = torch.from_numpy(complex_gaussian(op.N, 33, cols=2)).cuda()
    Yd = X @ (Z * F).T
    Y = far.apply(X)
    err = float(torch.linalg.norm(Y - Yd) / torch.linalg.norm(Yd))
    _say(f"  3 levels: {[(i['boxes'], i['far_pairs'], i['splines'], i['points_per_axis']) for i in infos]}; "
         f"vs dense far entries {err:.2e}")
    assert err <= 2e-3
    far.close()
    op.close()
