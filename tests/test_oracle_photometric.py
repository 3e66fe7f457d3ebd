"""Pins of the oracle's photometric loss, gradient and Gauss-Newton refinement (project extension
of the fitted similarity of Eq. 7 with the brightness constancy of Eq. 3).

Pinned against: closed forms on a linear ramp (bilinear sampling is exact there, so the loss, the
gradient and the Gauss-Newton terms are polynomials in theta computed here independently), exact zero
for an integer translation, central finite differences in binary64 at h = 1e-3 (1e-3 relative), the
parameter conversion from a fitted similarity, and recovery of a known sub-pixel translation.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1701_03572_amd import synth

ALPHA, BETA, GAMMA = 2.0, 3.0, 5.0


def ramp(w, h):
    y, x = np.mgrid[0:h, 0:w]
    img = ALPHA * x + BETA * y + GAMMA
    assert img.max() <= 255
    return img.astype(np.uint8)


def ramp_closed_form(theta, omega, w, h):
    cx, cy, rho = (w - 1) / 2.0, (h - 1) / 2.0, max(w, h) / 2.0
    x0, y0, x1, y1 = omega
    y, x = np.mgrid[y0:y1, x0:x1].astype(np.float64)
    dx, dy = (x - cx) / rho, (y - cy) / rho
    a, b, tx, ty = theta
    r = ALPHA * (a * dx - b * dy + tx) + BETA * (b * dx + a * dy + ty)
    J = np.stack([ALPHA * dx + BETA * dy, -ALPHA * dy + BETA * dx, np.full_like(dx, ALPHA), np.full_like(dx, BETA)])
    J = J.reshape(4, -1)
    r = r.ravel()
    return {"loss": float(r @ r), "grad": 2.0 * J @ r, "jtj": J @ J.T, "jtr": J @ r}


@pytest.mark.parametrize("theta", [(0.0, 0.0, 0.0, 0.0), (0.7, -0.4, 1.25, -0.5), (-1.5, 2.0, -0.3, 0.8)])
def test_ramp_closed_form(theta):
    w, h = 56, 40
    img = ramp(w, h)
    om = O.photo_omega(theta, w, h)
    got = O.photo_global(img, img, theta, om)
    ref = ramp_closed_form(theta, om, w, h)
    scale = max(ref["loss"], 1.0)
    assert abs(got["loss"] - ref["loss"]) <= 1e-10 * scale
    for k in ("grad", "jtr"):
        np.testing.assert_allclose(got[k], ref[k], rtol=1e-10, atol=1e-9 * math.sqrt(scale))
    np.testing.assert_allclose(got["jtj"], ref["jtj"], rtol=1e-12, atol=1e-13 * np.abs(ref["jtj"]).max())


def test_integer_translation_is_exact_zero():
    big = synth.smooth_random_image(200, 150, 4, sigma=1.5)
    tx, ty = 3, -2
    f0 = big[20:120, 20:180]
    f1 = big[20 + ty:120 + ty, 20 + tx:180 + tx]
    # f1[y, x] = big[y + 20 + ty, x + 20 + tx] = f0[y + ty, x + tx], so f1(x - t) = f0(x): T(x) = x - t
    theta = (0.0, 0.0, -float(tx), -float(ty))
    om = O.photo_omega(theta, 160, 100)
    got = O.photo_global(f0, f1, theta, om)
    assert got["loss"] == 0.0
    assert np.all(got["grad"] == 0.0) and np.all(got["jtr"] == 0.0)


def fd_global(f0, f1, theta, om, h=1e-3):
    g = np.zeros(4)
    for k in range(4):
        tp, tm = np.array(theta, float), np.array(theta, float)
        tp[k] += h
        tm[k] -= h
        g[k] = (O.photo_global(f0, f1, tp, om)["loss"] - O.photo_global(f0, f1, tm, om)["loss"]) / (2 * h)
    return g


@pytest.mark.parametrize("seed", [0, 1])
def test_global_gradient_matches_finite_differences(seed):
    rng = np.random.default_rng(seed)
    w, h = 160, 120
    f0 = synth.smooth_random_image(w, h, 10 + seed, sigma=2.0)
    f1 = O.warp(f0, [1.0, -0.01, 0.6, 0.01, 1.0, -0.3])
    theta = rng.normal(0, 0.5, 4)
    om = O.photo_omega(theta, w, h, extra=1)
    an = O.photo_global(f0, f1, theta, om)["grad"]
    fd = fd_global(f0, f1, theta, om)
    np.testing.assert_allclose(an, fd, rtol=1e-3, atol=1e-3 * np.abs(an).max())


def test_feature_ramp_closed_form():
    w, h = 56, 40
    img = ramp(w, h)
    u = np.array([[20.0, 15.0], [30.5, 20.25], [25.0, 18.0]])
    d = np.array([[0.3, -0.2], [-0.45, 0.1], [0.0, 0.0]])
    loss, grad = O.photo_feature(img, img, u, d, win_half=5)
    n = 11 * 11
    r = ALPHA * d[:, 0] + BETA * d[:, 1]
    np.testing.assert_allclose(loss, n * r * r, rtol=1e-12, atol=1e-10)
    np.testing.assert_allclose(grad, 2 * n * r[:, None] * np.array([ALPHA, BETA]), rtol=1e-12, atol=1e-10)


def test_feature_gradient_matches_finite_differences():
    rng = np.random.default_rng(3)
    w, h = 160, 120
    f0 = synth.smooth_random_image(w, h, 21, sigma=1.7)
    f1 = O.warp(f0, [1.0, 0.0, 0.8, 0.0, 1.0, -0.6])
    m = 60
    u = np.column_stack([rng.uniform(20, w - 20, m), rng.uniform(20, h - 20, m)])
    d = rng.normal(0, 0.6, (m, 2))
    hstep = 1e-3
    _, an = O.photo_feature(f0, f1, u, d)
    fd = np.zeros_like(an)
    for k in range(2):
        dp, dm = d.copy(), d.copy()
        dp[:, k] += hstep
        dm[:, k] -= hstep
        fd[:, k] = (O.photo_feature(f0, f1, u, dp)[0] - O.photo_feature(f0, f1, u, dm)[0]) / (2 * hstep)
    # every window sample shares the fractional offset of u + d: a component whose coordinate is within
    # 2h of an integer crosses a kink of the bilinear interpolant under the finite difference
    frac = (u + d) - np.floor(u + d)
    near = (frac < 2 * hstep) | (frac > 1 - 2 * hstep)
    ok = ~near
    assert ok.sum() >= 0.9 * ok.size
    scale = np.abs(an).max(axis=1, keepdims=True).repeat(2, axis=1)
    err = np.abs(an - fd) / np.maximum(np.abs(fd), 1e-3 * scale)
    assert err[ok].max() <= 1e-3, err[ok].max()


def test_theta_from_fit_reproduces_the_fitted_map():
    w, h = 640, 480
    a, b, tx, ty = 1.0123, -0.0171, 2.5, -1.75
    th = O.theta_from_fit((a, b, tx, ty), w, h)
    cx, cy, rho = O.photo_frame(w, h)
    rng = np.random.default_rng(7)
    p = rng.uniform(0, 640, (20, 2))
    xc, yc = p[:, 0] - cx, p[:, 1] - cy
    fit_x = a * xc - b * yc + tx + cx
    fit_y = b * xc + a * yc + ty + cy
    dx, dy = xc / rho, yc / rho
    tx_ = p[:, 0] + th[0] * dx - th[1] * dy + th[2]
    ty_ = p[:, 1] + th[1] * dx + th[0] * dy + th[3]
    np.testing.assert_allclose(tx_, fit_x, rtol=0, atol=1e-9)
    np.testing.assert_allclose(ty_, fit_y, rtol=0, atol=1e-9)


def test_refinement_recovers_subpixel_translation():
    w, h = 200, 150
    f0 = synth.smooth_random_image(w, h, 31, sigma=2.5)
    t = np.array([0.37, -0.21])
    # f1(x) = f0(x - t): the inverse-mapped warp by the translation t
    f1 = O.warp(f0, [1.0, 0.0, t[0], 0.0, 1.0, t[1]])
    theta0 = np.zeros(4)
    om = O.photo_omega(theta0, w, h, extra=3)
    th, (l0, l1), k = O.photo_refine(f0, f1, theta0, om, max_steps=5)
    assert k >= 1 and l1 < l0
    # T(x) = x + t maps f0 onto f1
    assert abs(th[2] - t[0]) < 0.03 and abs(th[3] - t[1]) < 0.03
    assert abs(th[0]) < 0.05 and abs(th[1]) < 0.05
