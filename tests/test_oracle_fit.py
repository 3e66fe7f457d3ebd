"""Pins of the oracle's robust rigid / similarity fit, hybrid switch and skip rule (Section 4,
Eq. 7; Section 4.1; the frame-skip rule of the motion-estimation workflow).

Pins: exact recovery of noise-free similarities and rigid motions; numpy.linalg.lstsq on the
2N x 4 design matrix; scipy's orthogonal Procrustes for the rigid model; the nesting invariant
E_s <= E_r; RANSAC removes planted outliers; published SplitMix64 outputs; the paper's Table 1
block totals equal the number of complete 20-pair dwell blocks of its Table 2 frame counts.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy.linalg import orthogonal_procrustes

from oracle import oracle as O

W, H = 640, 480
CX, CY = (W - 1) / 2.0, (H - 1) / 2.0
GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))


def sim_apply(p, pts):
    a, b, tx, ty = p
    x, y = pts[:, 0] - CX, pts[:, 1] - CY
    return np.stack([a * x - b * y + tx + CX, b * x + a * y + ty + CY], 1)


def fp(model, iters=0, seed=7, min_valid=10, dwell=20, thr=1.0):
    return O.fit_params(model, iters, thr, seed, 0, min_valid, dwell, W, H)


def rand_pts(n, seed):
    rng = np.random.default_rng(seed)
    return np.stack([rng.uniform(20, W - 20, n), rng.uniform(20, H - 20, n)], 1)


def test_splitmix64_published_outputs():
    # the first three outputs of SplitMix64 from state 0
    assert O.draw(0, 0, 0, 0, 0) == 0xE220A8397B1DCDAF
    assert O.draw(0, 0, 0, 0, 1) == 0x6E789E6AA1B965F4
    assert O.draw(0, 0, 0, 1, 0) == 0x06C45D188009454F


@pytest.mark.parametrize("iters", [0, 64])
def test_exact_similarity_recovery(iters):
    src = rand_pts(200, 1)
    true = (math.cos(0.03) * 1.01, math.sin(0.03) * 1.01, 4.25, -3.5)
    dst = sim_apply(true, src)
    p, info, inl = O.fit_pair(src, dst, None, fp(O.SIMILARITY, iters), 0)
    assert np.max(np.abs(p - true)) < 1e-10
    assert info["n_inliers"] == 200 and inl.all() and not info["skipped"]


@pytest.mark.parametrize("iters", [0, 64])
def test_exact_rigid_recovery(iters):
    src = rand_pts(150, 2)
    th = -0.02
    true = (math.cos(th), math.sin(th), -7.0, 2.75)
    dst = sim_apply(true, src)
    p, info, _ = O.fit_pair(src, dst, None, fp(O.RIGID, iters), 0)
    assert np.max(np.abs(p - true)) < 1e-10


def test_pure_translation():
    src = rand_pts(50, 3)
    rng = np.random.default_rng(4)
    dst = src + np.array([3.0, -1.5]) + rng.normal(0, 0.2, src.shape)
    p, _, _ = O.fit_pair(src, dst, None, fp(O.SIMILARITY, 0), 0)
    # no rotation/scale in the data would give a = 1, b = 0; with noise check translation
    dst_exact = src + np.array([3.0, -1.5])
    p2, _, _ = O.fit_pair(src, dst_exact, None, fp(O.SIMILARITY, 0), 0)
    assert abs(p2[0] - 1) < 1e-12 and abs(p2[1]) < 1e-12
    np.testing.assert_allclose(p2[2:], [3.0, -1.5], atol=1e-10)
    assert abs(p[2] - 3.0) < 0.2 and abs(p[3] + 1.5) < 0.2


def test_similarity_ls_equals_lstsq():
    src = rand_pts(120, 5)
    rng = np.random.default_rng(6)
    dst = sim_apply((0.99, 0.02, 1.0, 2.0), src) + rng.normal(0, 0.5, src.shape)
    p, _, _ = O.fit_pair(src, dst, None, fp(O.SIMILARITY, 0), 0)
    x, y = src[:, 0] - CX, src[:, 1] - CY
    u, v = dst[:, 0] - CX, dst[:, 1] - CY
    A = np.zeros((2 * len(x), 4))
    A[0::2] = np.stack([x, -y, np.ones_like(x), np.zeros_like(x)], 1)
    A[1::2] = np.stack([y, x, np.zeros_like(x), np.ones_like(x)], 1)
    rhs = np.empty(2 * len(x))
    rhs[0::2], rhs[1::2] = u, v
    ref = np.linalg.lstsq(A, rhs, rcond=None)[0]
    np.testing.assert_allclose(p, ref, rtol=1e-10, atol=1e-9)


def test_rigid_ls_equals_procrustes():
    src = rand_pts(80, 7)
    rng = np.random.default_rng(8)
    dst = sim_apply((math.cos(0.05) * 1.02, math.sin(0.05) * 1.02, -3, 5), src) + rng.normal(0, 0.4, src.shape)
    p, _, _ = O.fit_pair(src, dst, None, fp(O.RIGID, 0), 0)
    s = src - [CX, CY]
    d = dst - [CX, CY]
    ms, md = s.mean(0), d.mean(0)
    R, _ = orthogonal_procrustes(s - ms, d - md)          # (s - ms) @ R ~ (d - md)
    assert np.linalg.det(R) > 0
    th = math.atan2(R[0, 1], R[0, 0])
    assert abs(math.atan2(p[1], p[0]) - th) < 1e-10
    t = md - np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]]) @ ms
    np.testing.assert_allclose(p[2:], t, atol=1e-8)


@pytest.mark.parametrize("seed", range(5))
def test_similarity_never_worse_than_rigid_in_least_squares(seed):
    src = rand_pts(60, 10 + seed)
    rng = np.random.default_rng(20 + seed)
    dst = sim_apply((1.0 + rng.normal(0, 0.01), rng.normal(0, 0.02), 0, 0), src) + rng.normal(0, 1.0, src.shape)
    st = O.new_hybrid_state()
    _, info, _ = O.fit_pair(src, dst, None, fp(O.HYBRID, 0), 0, st)
    assert info["decided_here"] == 1
    assert info["err_sim"] <= info["err_rigid"] + 1e-12


def test_ransac_without_outliers_equals_ls():
    src = rand_pts(100, 30)
    rng = np.random.default_rng(31)
    dst = sim_apply((1.001, 0.01, 2, -1), src) + rng.normal(0, 0.05, src.shape)
    p0, _, _ = O.fit_pair(src, dst, None, fp(O.SIMILARITY, 0), 0)
    p1, info, inl = O.fit_pair(src, dst, None, fp(O.SIMILARITY, 128), 0)
    assert inl.all()
    np.testing.assert_array_equal(p0, p1)


@pytest.mark.parametrize("model", [O.SIMILARITY, O.RIGID])
def test_planted_outliers_are_excluded(model):
    src = rand_pts(300, 40)
    rng = np.random.default_rng(41)
    true = (math.cos(0.01), math.sin(0.01), 3, 1) if model == O.RIGID else (1.004, 0.012, 3, 1)
    dst = sim_apply(true, src) + rng.normal(0, 0.1, src.shape)
    bad = rng.random(300) < 0.35
    dst[bad] += rng.uniform(6, 30, (bad.sum(), 2)) * rng.choice([-1, 1], (bad.sum(), 2))
    p, info, inl = O.fit_pair(src, dst, None, fp(model, 128), 0)
    np.testing.assert_array_equal(inl.astype(bool), ~bad)
    assert np.max(np.abs(sim_apply(p, src[~bad]) - sim_apply(true, src[~bad]))) < 0.05


def test_skip_and_validity_mask():
    src = rand_pts(30, 50)
    dst = src + 1.0
    valid = np.zeros(30, np.uint8)
    valid[:9] = 1                                  # 9 < min_valid = 10
    p, info, inl = O.fit_pair(src, dst, valid, fp(O.SIMILARITY, 64), 0)
    assert info["skipped"] == 1 and info["n_valid"] == 9
    np.testing.assert_array_equal(p, [1, 0, 0, 0])
    valid[:10] = 1
    dst[20] += 100.0                               # invalid slots never influence the fit
    p, info, inl = O.fit_pair(src, dst, valid, fp(O.SIMILARITY, 64), 0)
    assert info["skipped"] == 0 and info["n_valid"] == 10
    np.testing.assert_allclose(p, [1, 0, 1, 1], atol=1e-10)
    assert inl[10:].sum() == 0


def decisions_over(n_frames, dwell=20, skip=()):
    src = rand_pts(12, 60)
    dst = src + 0.5
    st = O.new_hybrid_state()
    made = []
    for k in range(n_frames - 1):
        valid = np.zeros(12, np.uint8) if k in skip else None
        _, info, _ = O.fit_pair(src, dst, valid, fp(O.HYBRID, 0, dwell=dwell), k, st)
        if info["decided_here"]:
            made.append(k)
    return made


@pytest.mark.parametrize("video", sorted(GOLD["videos"]))
def test_table1_counts_equal_complete_dwell_blocks(video):
    v = GOLD["videos"][video]
    n = v["frames"]
    made = decisions_over(n, GOLD["dwell_frames"])
    n_pairs = n - 1
    complete = [k for k in made if k + GOLD["dwell_frames"] <= n_pairs]
    assert len(complete) == v["rigid_blocks"] + v["similarity_blocks"]
    assert len(made) == math.ceil(n_pairs / GOLD["dwell_frames"])
    assert all(k % 20 == 0 for k in made)


def test_decision_moves_to_first_unskipped_pair_of_block():
    made = decisions_over(61, 20, skip={20, 21, 40})
    assert made == [0, 22, 41]
