"""Pins of the oracle's 6-DOF affine candidate (Eq. 7-8: [A|t] minimising the squared residuals
over the point pairs; a later variant of the method, Section 4.1 keeps 4 DOF) and the three-way
hybrid built on it.

Pins: exact recovery of noise-free affine motions; numpy.linalg.lstsq on the 2N x 6 design of
Eq. 8; the exact solve through three points against numpy.linalg.solve; RANSAC removes planted
outliers (inlier set equal to the planted one, parameters equal to lstsq on it); collinear point
sets fall back to the similarity fit; the nesting invariant E_a <= E_s <= E_r of least squares; the
nearest similarity in the Frobenius norm against a least-squares projection; the three-way
hybrid's dwell blocks and choice rule; the affine draws' counters never meet the 2-point draws'.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O

W, H = 640, 480
CX, CY = (W - 1) / 2.0, (H - 1) / 2.0


def fp(model, iters=0, seed=7, min_valid=10, dwell=20, thr=1.0):
    return O.fit_params(model, iters, thr, seed, 0, min_valid, dwell, W, H)


def rand_pts(n, seed):
    rng = np.random.default_rng(seed)
    return np.stack([rng.uniform(20, W - 20, n), rng.uniform(20, H - 20, n)], 1)


def aff_apply(m, pts):
    """m = (a11, a12, tx, a21, a22, ty) in centred coordinates, applied to pixel coordinates."""
    x, y = pts[:, 0] - CX, pts[:, 1] - CY
    return np.stack([m[0] * x + m[1] * y + m[2] + CX, m[3] * x + m[4] * y + m[5] + CY], 1)


def design_lstsq(src, dst):
    """Least squares of Eq. 7 through the 2N x 6 design of Eq. 8 (rows [x y 1 0 0 0] and
    [0 0 0 x y 1]), centred coordinates."""
    x, y = src[:, 0] - CX, src[:, 1] - CY
    n = len(x)
    D = np.zeros((2 * n, 6))
    D[0::2, 0], D[0::2, 1], D[0::2, 2] = x, y, 1.0
    D[1::2, 3], D[1::2, 4], D[1::2, 5] = x, y, 1.0
    r = np.empty(2 * n)
    r[0::2], r[1::2] = dst[:, 0] - CX, dst[:, 1] - CY
    return np.linalg.lstsq(D, r, rcond=None)[0]


SHEAR = (1.02, 0.035, 4.5, -0.012, 0.975, -2.25)


@pytest.mark.parametrize("iters", [0, 64])
def test_exact_affine_recovery(iters):
    src = rand_pts(180, 1)
    dst = aff_apply(SHEAR, src)
    p4, m6, info, inl = O.fit_pair_affine(src, dst, None, fp(O.AFFINE, iters), 0)
    assert np.max(np.abs(m6 - SHEAR)) < 1e-10
    assert info["model"] == O.AFFINE and info["n_inliers"] == 180 and inl.all()


def test_least_squares_equals_design_lstsq():
    rng = np.random.default_rng(2)
    src = rand_pts(300, 2)
    dst = aff_apply(SHEAR, src) + rng.normal(0, 0.7, (300, 2))
    _, m6, info, _ = O.fit_pair_affine(src, dst, None, fp(O.AFFINE, 0), 0)
    ref = design_lstsq(src, dst)
    np.testing.assert_allclose(m6, ref, rtol=1e-9, atol=1e-9)


def test_three_points_give_the_exact_affine():
    src = np.array([[100.0, 80.0], [420.0, 130.0], [260.0, 390.0]])
    dst = src @ np.array([[0.97, 0.02], [-0.05, 1.04]]).T + [3.0, -6.0]
    _, m6, info, inl = O.fit_pair_affine(src, dst, None, fp(O.AFFINE, 16, min_valid=3), 0)
    # A [x y 1]^T = [x' y']^T for the three points, solved as one 6 x 6 system
    x, y = src[:, 0] - CX, src[:, 1] - CY
    M = np.zeros((6, 6))
    b = np.zeros(6)
    for i in range(3):
        M[2 * i, :3] = [x[i], y[i], 1.0]
        M[2 * i + 1, 3:] = [x[i], y[i], 1.0]
        b[2 * i], b[2 * i + 1] = dst[i, 0] - CX, dst[i, 1] - CY
    np.testing.assert_allclose(m6, np.linalg.solve(M, b), rtol=1e-9, atol=1e-9)
    assert inl.all() and info["n_inliers"] == 3


def test_planted_outliers_are_excluded():
    rng = np.random.default_rng(3)
    n = 400
    src = rand_pts(n, 3)
    dst = aff_apply(SHEAR, src) + rng.normal(0, 0.15, (n, 2))
    bad = rng.random(n) < 0.3
    dst[bad] += rng.uniform(8, 40, (bad.sum(), 2)) * rng.choice([-1, 1], (bad.sum(), 2))
    _, m6, info, inl = O.fit_pair_affine(src, dst, None, fp(O.AFFINE, 128), 0)
    np.testing.assert_array_equal(inl.astype(bool), ~bad)
    np.testing.assert_allclose(m6, design_lstsq(src[~bad], dst[~bad]), rtol=1e-9, atol=1e-9)
    assert info["n_inliers"] == (~bad).sum()


def test_collinear_points_fall_back_to_the_similarity():
    t = np.linspace(0, 1, 40)
    src = np.stack([60 + 500 * t, 50 + 300 * t], 1)
    rng = np.random.default_rng(4)
    dst = src * 1.01 + [2.0, -1.0] + rng.normal(0, 0.2, (40, 2))
    p4, m6, info, _ = O.fit_pair_affine(src, dst, None, fp(O.AFFINE, 0), 0)
    ps, _, _ = O.fit_pair(src, dst, None, fp(O.SIMILARITY, 0), 0)
    np.testing.assert_array_equal(m6, [ps[0], -ps[1], ps[2], ps[1], ps[0], ps[3]])
    np.testing.assert_allclose(p4, ps, rtol=0, atol=1e-15)


@pytest.mark.parametrize("seed", [5, 6, 7])
def test_nesting_and_three_way_choice(seed):
    rng = np.random.default_rng(seed)
    src = rand_pts(250, seed)
    m = (1.0 + rng.normal(0, 0.02), rng.normal(0, 0.03), 3.0, rng.normal(0, 0.03), 1.0 + rng.normal(0, 0.02), 1.0)
    dst = aff_apply(m, src) + rng.normal(0, 0.5, (250, 2))
    _, m6, info, _ = O.fit_pair_affine(src, dst, None, fp(O.HYBRID3, 0), 0)
    er, es, ea = info["err_rigid"], info["err_sim"], info["err_affine"]
    assert ea <= es * (1 + 1e-12) and es <= er * (1 + 1e-12)
    # the RMS over all points, recomputed from the design solution
    ref = design_lstsq(src, dst)
    res = aff_apply(ref, src) - dst
    assert ea == pytest.approx(math.sqrt(np.mean(np.sum(res ** 2, 1))), rel=1e-9)
    best = O.RIGID if er < es else O.SIMILARITY
    expect = O.AFFINE if ea < (er if best == O.RIGID else es) else best
    assert info["model"] == expect and info["decided_here"] == 1


def test_nearest_similarity_of_an_affine_result():
    src = rand_pts(100, 8)
    dst = aff_apply(SHEAR, src)
    p4, m6, _, _ = O.fit_pair_affine(src, dst, None, fp(O.AFFINE, 0), 0)
    # least-squares projection of A onto {[[a, -b], [b, a]]}: 4 equations in (a, b)
    A = np.array([[m6[0], m6[1]], [m6[3], m6[4]]])
    G = np.array([[1.0, 0.0], [0.0, -1.0], [0.0, 1.0], [1.0, 0.0]])
    ab = np.linalg.lstsq(G, A.reshape(-1), rcond=None)[0]
    np.testing.assert_allclose(p4[:2], ab, rtol=1e-12, atol=1e-15)
    assert p4[2] == m6[2] and p4[3] == m6[5]


def test_three_way_dwell_blocks_and_skips():
    src = rand_pts(30, 9)
    dst = aff_apply(SHEAR, src) + np.random.default_rng(9).normal(0, 0.3, (30, 2))
    st = O.new_hybrid_state()
    made, models = [], []
    for k in range(61):
        valid = np.zeros(30, np.uint8) if k in (20, 21, 40) else None
        _, m6, info, _ = O.fit_pair_affine(src, dst, valid, fp(O.HYBRID3, 32), k, st)
        if info["decided_here"]:
            made.append(k)
        models.append(info["model"])
        if k in (20, 21, 40):
            assert info["skipped"] and np.array_equal(m6, [1, 0, 0, 0, 1, 0])
    assert made == [0, 22, 41, 60]
    assert set(models) == {O.AFFINE}


def test_affine_draw_counters_are_disjoint_from_two_point_draws():
    # SplitMix64 is a bijection of its counter, so distinct counters give distinct outputs
    two = {O.draw(99, 3, 17, h, k) for h in range(8191) for k in range(2)}
    three = {O.draw3(99, 3, 17, h, k) for h in range(8191) for k in range(3)}
    assert len(two) == 2 * 8191 and len(three) == 3 * 8191
    assert not (two & three)
