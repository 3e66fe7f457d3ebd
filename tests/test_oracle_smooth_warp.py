"""Pins of the oracle's trajectory smoothing (Section 5.1, Section 6) and warp (Section 5).

Smoothing pins: constant and linear trajectories, closed-form window means of j^2 with truncated
ends (centred and causal windows), the causal correction -r v of a constant pan, causality (later
pairs never change earlier outputs), the global mean when the radius covers the sequence, the Kalman steady-state gain of a
random walk (Riccati fixed point), and the correction matrix of a pure translation.
Warp pins: identity, integer shifts with zero fill, the 180 degree rotation as a flip, half-pixel
shifts, and scipy's map_coordinates (order 1, grid-constant) on general similarities.
"""
import math

import numpy as np
import pytest
from scipy import ndimage

from oracle import oracle as O
from paper_1701_03572_amd import synth

W, H = 320, 240


def pairs_const(n, a=1.0, b=0.0, tx=0.0, ty=0.0):
    return np.tile([a, b, tx, ty], (n - 1, 1)).astype(np.float64)


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_identity_pairs_give_identity_matrices(mode):
    n = 40
    _, _, mats = O.smooth(pairs_const(n), n, mode, 7, 0.05, 0.0, W, H)
    np.testing.assert_array_equal(mats, np.tile([1, 0, 0, 0, 1, 0], (n, 1)))


def test_linear_trajectory_has_no_interior_correction():
    n, r = 50, 6
    _, sm, mats = O.smooth(pairs_const(n, tx=1.5, ty=-0.25), n, 0, r, 0.0, 0.0, W, H)
    traj = np.arange(n)[:, None] * np.array([1.5, -0.25])
    for j in range(r, n - r):
        np.testing.assert_allclose(sm[j, :2], traj[j], atol=1e-12)
        np.testing.assert_allclose(mats[j], [1, 0, 0, 0, 1, 0], atol=1e-12)


def test_window_means_of_squares_with_truncated_ends():
    n, r = 30, 4
    # tx of pair k = 2k + 1 makes the trajectory P_j = j^2
    pp = np.array([[1.0, 0.0, 2.0 * k + 1.0, 0.0] for k in range(n - 1)])
    traj, sm, _ = O.smooth(pp, n, 0, r, 0.0, 0.0, W, H)
    np.testing.assert_allclose(traj[:, 0], np.arange(n) ** 2.0, atol=0)

    def s2(m):                                    # sum_{i=0}^{m} i^2
        return m * (m + 1) * (2 * m + 1) / 6.0

    for j in range(n):
        lo, hi = max(0, j - r), min(n - 1, j + r)
        mean = (s2(hi) - (s2(lo - 1) if lo > 0 else 0.0)) / (hi - lo + 1)
        assert abs(sm[j, 0] - mean) <= 1e-12 * max(1.0, mean)


@pytest.mark.parametrize("r", [1, 4, 7])
def test_causal_window_of_a_constant_pan(r):
    """Causal mode (the sliding store of the real-time version, Section 6) averages P over
    [max(0, j - 2r), j]. With a constant pan v, P_j = j v: the mean is (j - r) v once j >= 2r, so the
    correction is exactly -r v there, and j v / 2 over the truncated window before it."""
    n = 40
    v = np.array([1.5, -0.25])
    _, sm, mats = O.smooth(pairs_const(n, tx=v[0], ty=v[1]), n, 1, r, 0.0, 0.0, W, H)
    for j in range(n):
        want = (j - r) * v if j >= 2 * r else j * v / 2.0
        np.testing.assert_allclose(sm[j, :2], want, rtol=0, atol=1e-12 * max(1.0, j))
        np.testing.assert_allclose(mats[j], [1, 0, want[0] - j * v[0], 0, 1, want[1] - j * v[1]], rtol=0,
                                   atol=1e-12 * max(1.0, j))


@pytest.mark.parametrize("r", [2, 5])
def test_causal_window_means_of_squares(r):
    """P_j = j^2: the causal mean over [lo, j], lo = max(0, j - 2r), is (S(j) - S(lo - 1)) / (j - lo + 1)
    with S(m) = m (m + 1) (2m + 1) / 6."""
    n = 30
    pp = np.array([[1.0, 0.0, 2.0 * k + 1.0, 0.0] for k in range(n - 1)])
    _, sm, _ = O.smooth(pp, n, 1, r, 0.0, 0.0, W, H)

    def s2(m):
        return m * (m + 1) * (2 * m + 1) / 6.0

    for j in range(n):
        lo = max(0, j - 2 * r)
        mean = (s2(j) - (s2(lo - 1) if lo > 0 else 0.0)) / (j - lo + 1)
        assert abs(sm[j, 0] - mean) <= 1e-12 * max(1.0, mean)


def test_causal_output_ignores_later_pairs():
    """Frame j's causal output depends on pairs before j only: changing pair k leaves frames <= k
    unchanged (a centred or off-by-one window would not)."""
    n, r = 24, 3
    rng = np.random.default_rng(4)
    pp = np.stack([np.ones(n - 1), np.zeros(n - 1), rng.normal(0, 3, n - 1), rng.normal(0, 3, n - 1)], 1)
    _, sm, mats = O.smooth(pp, n, 1, r, 0.0, 0.0, W, H)
    for k in (0, 7, 15):
        q = pp.copy()
        q[k, 2] += 5.0
        _, sm2, mats2 = O.smooth(q, n, 1, r, 0.0, 0.0, W, H)
        np.testing.assert_array_equal(sm2[:k + 1], sm[:k + 1])
        np.testing.assert_array_equal(mats2[:k + 1], mats[:k + 1])
        assert np.all(sm2[k + 1:k + 2 * r + 2, 0] != sm[k + 1:k + 2 * r + 2, 0])


def test_radius_beyond_sequence_is_global_mean():
    n = 12
    rng = np.random.default_rng(1)
    pp = np.stack([np.ones(n - 1), np.zeros(n - 1), rng.normal(0, 3, n - 1), rng.normal(0, 3, n - 1)], 1)
    traj, sm, _ = O.smooth(pp, n, 0, 100, 0.0, 0.0, W, H)
    for j in range(n):
        np.testing.assert_allclose(sm[j], traj.mean(0), atol=1e-12)


@pytest.mark.parametrize("rho", [0.02, 0.5, 3.0])
def test_kalman_steady_state_gain(rho):
    n, m = 400, 300
    pp = pairs_const(n)
    pp[m - 1, 2] = 1.0                            # a unit step of the trajectory at frame m
    _, sm, _ = O.smooth(pp, n, 2, 0, rho, 0.0, W, H)
    # predicted covariance at the fixed point of S <- (S + rho) / (S + rho + 1), and its gain
    p_inf = (rho + math.sqrt(rho * rho + 4 * rho)) / 2.0
    k_inf = p_inf / (p_inf + 1.0)
    assert abs(sm[m, 0] - k_inf) < 1e-12
    assert abs(sm[m - 1, 0]) == 0.0


def test_kalman_huge_process_noise_follows_trajectory():
    n = 30
    rng = np.random.default_rng(2)
    pp = np.stack([np.ones(n - 1), np.zeros(n - 1), rng.normal(0, 3, n - 1), rng.normal(0, 3, n - 1)], 1)
    traj, sm, _ = O.smooth(pp, n, 2, 0, 1e12, 0.0, W, H)
    np.testing.assert_allclose(sm, traj, atol=1e-9)


def test_translation_correction_matrix_and_rotation_about_centre():
    n = 3
    pp = np.array([[1.0, 0.0, 4.0, -2.0], [1.0, 0.0, -4.0, 2.0]])
    traj, sm, mats = O.smooth(pp, n, 0, 5, 0.0, 0.0, W, H)
    # global mean of positions (0,0), (4,-2), (0,0) is (4/3, -2/3)
    np.testing.assert_allclose(mats[1], [1, 0, 4 / 3 - 4, 0, 1, -2 / 3 + 2], atol=1e-12)
    # a pure rotation correction keeps the image centre fixed
    th = 0.1
    pp = np.array([[math.cos(th), math.sin(th), 0.0, 0.0], [1.0, 0.0, 0.0, 0.0]])
    _, _, mats = O.smooth(pp, 3, 0, 5, 0.0, 0.0, W, H)
    M = mats[0].reshape(2, 3)
    c = np.array([(W - 1) / 2, (H - 1) / 2, 1.0])
    np.testing.assert_allclose(M @ c, c[:2], atol=1e-9)
    # angles 0, th, th: mean 2 th / 3, so frame 0 is corrected by 2 th / 3
    assert abs(math.atan2(M[1, 0], M[0, 0]) - 2 * th / 3) < 1e-12


def test_crop_zoom_about_centre():
    _, _, mats = O.smooth(pairs_const(2), 2, 0, 1, 0, 0.1, W, H)
    M = mats[0].reshape(2, 3)
    np.testing.assert_allclose(M[:, :2], np.eye(2) / 0.8, atol=1e-15)
    c = np.array([(W - 1) / 2, (H - 1) / 2, 1.0])
    np.testing.assert_allclose(M @ c, c[:2], atol=1e-12)


# ------------------------------------------------------------------------------------------- warp

def test_identity_warp_is_exact():
    img = synth.random_image(W, H, 1)
    np.testing.assert_array_equal(O.warp(img, [1, 0, 0, 0, 1, 0]), img)


@pytest.mark.parametrize("t", [(3, -5), (-17, 8), (0, 1)])
def test_integer_shift_with_zero_fill(t):
    img = synth.random_image(W, H, 2)
    out = O.warp(img, [1, 0, t[0], 0, 1, t[1]], border=0)
    ref = np.zeros_like(img)
    tx, ty = t
    ref[max(0, ty):H + min(0, ty), max(0, tx):W + min(0, tx)] = img[max(0, -ty):H - max(0, ty),
                                                                    max(0, -tx):W - max(0, tx)]
    np.testing.assert_array_equal(out, ref)


def test_half_turn_about_centre_is_a_flip():
    img = synth.random_image(W, H, 3)
    out = O.warp(img, [-1, 0, W - 1, 0, -1, H - 1])
    np.testing.assert_array_equal(out, img[::-1, ::-1])


def test_half_pixel_shift_rounds_half_up():
    img = synth.random_image(W, H, 4)
    out = O.warp(img, [1, 0, -0.5, 0, 1, 0])       # output x samples source x + 0.5
    p = img[:, :-1].astype(np.int32)
    q = img[:, 1:].astype(np.int32)
    np.testing.assert_array_equal(out[:, :-1], ((p + q + 1) >> 1).astype(np.uint8))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_general_similarity_matches_scipy(seed):
    rng = np.random.default_rng(seed)
    img = synth.smooth_random_image(W, H, 10 + seed, sigma=1.2)
    th, s = rng.normal(0, 0.05), 1 + rng.normal(0, 0.02)
    a, b = s * math.cos(th), s * math.sin(th)
    M = np.array([[a, -b, rng.normal(0, 8)], [b, a, rng.normal(0, 8)]])
    out = O.warp(img, M.ravel(), border=0)
    Mi = np.linalg.inv(np.vstack([M, [0, 0, 1]]))[:2]
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    sx = Mi[0, 0] * xx + Mi[0, 1] * yy + Mi[0, 2]
    sy = Mi[1, 0] * xx + Mi[1, 1] * yy + Mi[1, 2]
    v = ndimage.map_coordinates(img.astype(np.float64), [sy, sx], order=1, mode="grid-constant", cval=0.0)
    ref = np.clip(np.floor(v + 0.5), 0, 255).astype(np.int32)
    d = np.abs(out.astype(np.int32) - ref)
    assert d.max() <= 1
    assert (d > 0).mean() < 1e-3
