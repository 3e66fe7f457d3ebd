"""Pins of the oracle's pyramidal Lucas-Kanade tracker with the backward check (Section 3.2,
Eqs. 3-6; Section 4.1 weeding).

Pins: zero motion is a fixed point; integer translations by multiples of 2^(L-1) are recovered
(the pyramids shift exactly); one Gauss-Newton step equals numpy's least-squares solution of the
linearised constraint fx u + fy v + ft = 0 built with numpy.gradient; smooth sub-pixel shifts
are recovered; the backward error is that of a separate backward track.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1701_03572_amd import synth


def smooth_texture(w, h, dx=0.0, dy=0.0, seed=0):
    """Analytic band-limited texture sampled at (x - dx, y - dy), quantised to uint8."""
    rng = np.random.default_rng(seed)
    y, x = np.mgrid[0:h, 0:w].astype(np.float64)
    v = np.full((h, w), 128.0)
    for _ in range(24):
        f = rng.uniform(0.02, 0.12)
        th = rng.uniform(0, 2 * math.pi)
        ph = rng.uniform(0, 2 * math.pi)
        v += 9.0 * np.cos(2 * math.pi * f * (math.cos(th) * (x - dx) + math.sin(th) * (y - dy)) + ph)
    return np.clip(np.floor(v + 0.5), 0, 255).astype(np.uint8)


def test_zero_motion_is_exact():
    img = synth.smooth_random_image(160, 120, 1, sigma=2.0)
    pyr = O.pyramid(img, 3)
    pts = synth.random_points(40, 160, 120, 12, 2)
    out, st, fe, it = O.track_lk(pyr, pyr, pts)
    np.testing.assert_array_equal(out, pts)
    assert st.all()
    np.testing.assert_array_equal(fe, 0.0)
    assert (it == 1).all()


@pytest.mark.parametrize("t", [(16, -32), (-48, 16), (0, 0)])
def test_integer_translation_by_pyramid_multiple(t):
    L = 5
    big = synth.smooth_random_image(640, 480, 7, sigma=2.5)
    tx, ty = t
    x0, y0 = 120, 100
    a = big[y0:y0 + 256, x0:x0 + 320]
    b = big[y0 - ty:y0 - ty + 256, x0 - tx:x0 - tx + 320]      # b(x) = a(x - t): content moves by +t
    pa, pb = O.pyramid(a, L), O.pyramid(b, L)
    pts = synth.random_points(30, 320, 256, 0, 3)
    pts = pts[(pts[:, 0] > 110) & (pts[:, 0] < 210) & (pts[:, 1] > 100) & (pts[:, 1] < 156)]
    out, st, fe, it = O.track_lk(pa, pb, pts, win_half=10, max_iter=30, eps=1e-3)
    assert st.all()
    assert np.max(np.abs(out - (pts + np.array(t, np.float64)))) < 2e-3
    assert np.max(fe) < 4e-3


def test_one_step_equals_least_squares():
    img0 = synth.smooth_random_image(96, 80, 11, sigma=2.0)
    img1 = smooth_texture(96, 80, 0.4, -0.3, seed=4)        # any second image: one linear step
    u = np.array([[47.0, 38.0]])
    out, st, _, _ = O.track_lk([img0], [img1], u, win_half=10, max_iter=1, eps=0.0, fb=False)
    # linearised constraint over the 21x21 window at an integer point: samples are pixels,
    # gradients are central differences (numpy.gradient in the interior)
    f0 = img0.astype(np.float64)
    gy, gx = np.gradient(f0)
    sl = (slice(38 - 10, 38 + 11), slice(47 - 10, 47 + 11))
    Amat = np.stack([gx[sl].ravel(), gy[sl].ravel()], 1)
    rhs = (f0[sl] - img1.astype(np.float64)[sl]).ravel()
    eta = np.linalg.lstsq(Amat, rhs, rcond=None)[0]
    np.testing.assert_allclose(out[0] - u[0], eta, rtol=1e-9, atol=1e-12)


@pytest.mark.parametrize("shift", [(0.3, -0.7), (2.45, 1.2), (-5.6, 3.3)])
def test_subpixel_shift_of_smooth_texture(shift):
    a = smooth_texture(200, 160, 0, 0, seed=9)
    b = smooth_texture(200, 160, shift[0], shift[1], seed=9)
    pts = synth.random_points(25, 200, 160, 40, 5)
    out, st, fe, _ = O.track_lk(O.pyramid(a, 3), O.pyramid(b, 3), pts)
    assert st.all()
    err = out - pts - np.array(shift)
    assert np.max(np.abs(err)) < 0.05


def test_flat_window_is_lost():
    flat = np.full((120, 160), 100, np.uint8)
    pts = np.array([[80.0, 60.0]])
    out, st, _, _ = O.track_lk(O.pyramid(flat, 3), O.pyramid(flat, 3), pts)
    assert st[0] == 0


def test_dead_slots_are_not_tracked():
    img = synth.smooth_random_image(160, 120, 1, sigma=2.0)
    pyr = O.pyramid(img, 3)
    pts = synth.random_points(10, 160, 120, 12, 2)
    alive = np.array([1, 0] * 5, np.uint8)
    out, st, fe, _ = O.track_lk(pyr, pyr, pts, alive)
    np.testing.assert_array_equal(st, alive)
    assert np.isnan(fe[alive == 0]).all()


def test_backward_error_is_a_separate_backward_track():
    """fb_err is the distance from u of an independent next -> prev track started at v, and the
    status keeps exactly the forward-valid points within the threshold."""
    a = synth.smooth_random_image(200, 160, 21, sigma=1.5)
    b = smooth_texture(200, 160, 1.7, -2.2, seed=3)
    pa, pb = O.pyramid(a, 3), O.pyramid(b, 3)
    pts = synth.random_points(60, 200, 160, 30, 6)
    fwd, st_f, _, _ = O.track_lk(pa, pb, pts, fb=False)
    bwd, st_b, _, _ = O.track_lk(pb, pa, fwd, alive=st_f, fb=False)
    for thr in (0.05, 1.0, 1e9):
        _, st, fe, _ = O.track_lk(pa, pb, pts, fb=True, fb_thresh=thr)
        ok = st_f.astype(bool)
        d = np.hypot(*(bwd - pts).T)
        np.testing.assert_allclose(fe[ok], d[ok], rtol=0, atol=1e-12)
        np.testing.assert_array_equal(st.astype(bool), ok & st_b.astype(bool) & (d <= thr))


def test_eigen_margin_is_the_window_tensor_minimum_eigenvalue():
    """The reported margin of a single-level zero-motion track is |lambda_min(G) / 441 - tau| / tau
    with G the gradient tensor of the 21x21 window, here from numpy.gradient and numpy.linalg.eigvalsh
    (both passes see the same window at an integer point)."""
    img = synth.smooth_random_image(96, 80, 13, sigma=2.0)
    pts = np.array([[47.0, 38.0], [30.0, 25.0], [60.0, 50.0]])
    tau = 0.5
    _, st, _, _, mg = O.track_lk([img], [img], pts, min_eig=tau, with_margin=True)
    gy, gx = np.gradient(img.astype(np.float64))
    for i, (x, y) in enumerate(pts.astype(int)):
        sl = (slice(y - 10, y + 11), slice(x - 10, x + 11))
        G = np.array([[np.sum(gx[sl] ** 2), np.sum(gx[sl] * gy[sl])], [np.sum(gx[sl] * gy[sl]), np.sum(gy[sl] ** 2)]])
        lam = np.linalg.eigvalsh(G)[0] / 441.0
        assert abs(mg[i] - abs(lam - tau) / tau) <= 1e-9 * max(1.0, abs(lam - tau) / tau)
        assert st[i] == (lam >= tau)


def test_eigen_margin_is_the_smallest_over_levels_and_passes():
    """Moving the threshold onto one level's statistic drives the margin to zero; a dead slot, which
    runs no test, reports +inf."""
    a = synth.smooth_random_image(200, 160, 21, sigma=1.5)
    b = smooth_texture(200, 160, 1.7, -2.2, seed=3)
    pa, pb = O.pyramid(a, 3), O.pyramid(b, 3)
    pts = synth.random_points(20, 200, 160, 30, 6)
    _, _, _, _, m1 = O.track_lk(pa, pb, pts, min_eig=1.0, with_margin=True)
    # with tau' = tau (1 - m) or tau (1 + m) one of the statistics seen equals the new threshold
    for i in range(3):
        for tau in (1.0 * (1.0 - m1[i]), 1.0 * (1.0 + m1[i])):
            if tau <= 0:
                continue
            _, _, _, _, m2 = O.track_lk(pa, pb, pts[i:i + 1], min_eig=tau, with_margin=True)
            # either the statistic sits exactly on the new threshold, or the other sign was the hit
            if m2[0] < 1e-9:
                break
        else:
            raise AssertionError("no level statistic at distance %g" % m1[i])
    _, _, _, _, m3 = O.track_lk(pa, pb, pts[:2], alive=np.array([0, 1], np.uint8), with_margin=True)
    assert np.isinf(m3[0]) and np.isfinite(m3[1])
