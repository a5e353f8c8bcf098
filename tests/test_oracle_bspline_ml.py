"""Pins of the multilevel B-spline oracle (Sec. III-C, IV): the knot-insertion
transfer between levels is exact (the spline identity at random points, and
the paper's own check of Sec. IV-E: parent moments by quadrature against the
transferred child moments), the FFT translation equals the point-by-point
product, the interaction lists cover every pair of far leaf boxes exactly once,
one level reduces to the single-level oracle, and the multilevel far field
approaches the dense oracle's far entries."""
import numpy as np
import pytest

from oracle import bspline as bs
from oracle import cfill
from oracle.mesh import rwg_table
from paper_2606_13482_amd.inputs import icosphere


@pytest.mark.parametrize("s,p,sb,increase", [(8, 3, 2, False), (8, 3, 2, True), (6, 3, 1, False), (9, 5, 2, True),
                                             (7, 3, 0, False)])
def test_restriction_matrix_exact(s, p, sb, increase):
    """b_j^parent = sum_i C[j, i] b_i^child on each child's buffered interval,
    for both children, constant (Sec. IV-C) and doubled (Sec. IV-D) spline
    counts; the entries are convex weights (knot insertion keeps them in [0, 1])."""
    child = bs.BoxSplines(s, p, sb)
    parent = bs.BoxSplines(2 * s - p, p, sb) if increase else bs.BoxSplines(s, p, -(-sb // 2))
    rng = np.random.default_rng(2)
    for c, C in enumerate(bs.transfer_matrices(child, parent)):
        u_ch = 0.5 * c + 0.5 * child.u_eq
        x = rng.uniform(u_ch[0], u_ch[-1], 400)
        lhs = bs.basis(parent.u_eq, p, x)
        rhs = bs.basis(u_ch, p, x) @ C.T
        assert np.max(np.abs(lhs - rhs)) < 1e-13, (c, np.max(np.abs(lhs - rhs)))
        assert C.min() >= -1e-15 and C.max() <= 1 + 1e-15
        # parent splines without support on the child's interval have zero rows
        for j in range(C.shape[0]):
            lo, hi = parent.u_eq[j], parent.u_eq[j + p + 1]
            if hi <= u_ch[0] or lo >= u_ch[-1]:
                assert not np.any(C[j]), j


def test_restriction_requires_nested_knots():
    child = bs.BoxSplines(8, 3, 1)
    parent = bs.BoxSplines(9, 3, 1)       # spacing 1/6 against the child's 1/10: not nested
    with pytest.raises(ValueError):
        bs.transfer_matrices(child, parent)


@pytest.fixture(scope="module")
def sphere3():
    V, T = icosphere(3)
    return rwg_table(V, T)


def test_transfer_of_moments_sec_ivE(sphere3):
    """The paper's check of the interlevel transfer (Sec. IV-E): moments of the
    functions of each leaf box with the parent box's splines, by quadrature,
    against the child moments moved up by the transfer matrices: relative error
    at rounding level (1e-13), for the constant and the doubled spline count."""
    rwg = sphere3
    a = 0.35
    idx, lo, prot, origin = bs.box_level(rwg, a)
    for k, s in ((2.0, 8), (12.0, 8)):
        sb = bs.buffer_knots(prot, s, 3)
        cfg = bs.level_configs(s, 3, sb, a, 2, k)
        assert (cfg[1].s == s) == (k == 2.0)
        m_child = bs.moments(rwg, cfg[0], a, lo, transformed=False)
        par_idx = idx >> 1
        lo_par = origin + par_idx * (2 * a)
        m_par = bs.moments(rwg, cfg[1], 2 * a, lo_par, transformed=False)
        Cm = bs.transfer_matrices(cfg[0], cfg[1])
        worst = 0.0
        for m in range(0, rwg["N"], 7):
            c = idx[m] & 1
            mv = bs.apply3(Cm[c[0]], Cm[c[1]], Cm[c[2]], m_child[m])
            worst = max(worst, np.max(np.abs(mv - m_par[m])) / np.max(np.abs(m_par[m])))
        assert worst < 1e-13, (k, worst)


def test_fft_translation_equals_direct():
    """The FFT form of a translation (the three-level Toeplitz structure of G,
    Sec. III-C) equals G sampled point by point, for several box offsets."""
    sp = bs.BoxSplines(8, 3, 2)
    rng = np.random.default_rng(4)
    Mt = rng.standard_normal((2, 4) + (sp.n_st,) * 3) + 1j * rng.standard_normal((2, 4) + (sp.n_st,) * 3)
    a, k = 0.35, 2.0
    for off in ((2, 0, 0), (3, -2, 1), (-2, 2, -2), (5, 1, -4)):
        o = np.array(off, float) * a
        K = bs.translation_kernel(sp, a, o, k)
        yf = bs.translate_fft(K, Mt)
        yd = bs.translate_direct(sp, a, o, np.zeros(3), k, Mt)
        assert np.max(np.abs(yf - yd)) < 1e-12 * np.max(np.abs(yd)), off


def test_interaction_lists_partition():
    """Over the levels, every pair of far leaf boxes is translated exactly once
    (at the level where its ancestors are far and their parents near, or at the
    top level) and no near pair is."""
    rng = np.random.default_rng(5)
    leaf = np.unique(rng.integers(0, 16, size=(300, 3)), axis=0)
    for levels in (1, 2, 3):
        boxes0, lists = bs.interaction_lists(leaf, levels)
        count = np.zeros((len(boxes0), len(boxes0)), int)
        for l, L in enumerate(lists):
            anc = np.unique(np.concatenate([L["boxes"], boxes0 >> l]), axis=0, return_inverse=True)[1].ravel()[
                len(L["boxes"]):]
            pair = np.zeros((len(L["boxes"]), len(L["boxes"])), int)
            pair[L["pairs"][:, 0], L["pairs"][:, 1]] = 1
            count += pair[anc][:, anc]
        far = np.max(np.abs(boxes0[:, None, :] - boxes0[None, :, :]), axis=2) > 1
        assert np.array_equal(count, far.astype(int)), levels


@pytest.fixture(scope="module")
def dense3(sphere3):
    return cfill.fill(sphere3, 2.0)


def test_one_level_is_single_level(sphere3):
    """With one level the multilevel scheme is the single-level far field of
    Sec. III (moments aggregated before or after the transformation)."""
    rng = np.random.default_rng(6)
    x = rng.standard_normal(sphere3["N"]) + 1j * rng.standard_normal(sphere3["N"])
    y1, _ = bs.far_product(sphere3, 2.0, x, 0.7, 6, 3)
    y2, _ = bs.ml_far_product(sphere3, 2.0, x, 0.7, 1, 6, 3)
    assert np.linalg.norm(y1 - y2) < 1e-12 * np.linalg.norm(y1)


def test_two_levels_against_dense(sphere3, dense3):
    """Two levels (boxes of 0.35 m and 0.7 m on the 1920-unknown sphere, k = 2,
    cubic splines, s = 8): the multilevel far field against the dense oracle's
    entries between far leaf boxes, within 2e-3; the FFT and the point-by-point
    translations agree."""
    rng = np.random.default_rng(7)
    x = rng.standard_normal(sphere3["N"]) + 1j * rng.standard_normal(sphere3["N"])
    y, info = bs.ml_far_product(sphere3, 2.0, x, 0.35, 2, 8, 3)
    F = bs.leaf_far_mask(info["leaf_of"], info["leaf_boxes"])
    yd = (dense3 * F) @ x
    err = np.linalg.norm(y - yd) / np.linalg.norm(yd)
    assert err < 2e-3, err
    assert [len(L["pairs"]) for L in info["lists"]] == [5256, 386]
