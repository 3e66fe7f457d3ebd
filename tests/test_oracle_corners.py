"""Pins of the oracle's Shi-Tomasi detector (Section 3.1, Eq. 2: R = min(lambda1, lambda2);
corner budget; reduced region of interest).

The response is checked against scipy's Sobel filter + box sums + numpy's symmetric
eigensolver; the selection against analytic corner locations and the defining properties of a
greedy minimum-distance selection in the stated total order.
"""
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st
from scipy import ndimage

from oracle import oracle as O
from paper_1701_03572_amd import synth


def library_min_eig(img, rect):
    f = img.astype(np.float64)
    gx = ndimage.sobel(f, axis=1, mode="nearest")
    gy = ndimage.sobel(f, axis=0, mode="nearest")
    box = np.ones((3, 3))
    A = ndimage.correlate(gx * gx, box, mode="nearest")
    B = ndimage.correlate(gx * gy, box, mode="nearest")
    Cc = ndimage.correlate(gy * gy, box, mode="nearest")
    x0, y0, x1, y1 = rect
    T = np.stack([np.stack([A, B], -1), np.stack([B, Cc], -1)], -2)[y0:y1, x0:x1]
    return np.linalg.eigvalsh(T)[..., 0], A[y0:y1, x0:x1], B[y0:y1, x0:x1], Cc[y0:y1, x0:x1]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_min_eig_matches_eigvalsh(seed):
    img = synth.smooth_random_image(80, 64, seed, sigma=1.5)
    rect = (2, 2, 78, 62)
    lam = O.min_eig_map(img, rect)
    ref, A, B, Cc = library_min_eig(img, rect)
    T = O.tensor_map(img, rect)
    np.testing.assert_array_equal(T[..., 0], A.astype(np.int64))
    np.testing.assert_array_equal(T[..., 1], B.astype(np.int64))
    np.testing.assert_array_equal(T[..., 2], Cc.astype(np.int64))
    scale = np.maximum(A + Cc, 1.0)
    assert np.max(np.abs(lam - ref) / scale) < 1e-12
    assert (lam >= 0).all()


@settings(max_examples=25, deadline=None)
@given(seed=st.integers(0, 2**31 - 1))
def test_min_eig_random_noise(seed):
    img = synth.random_image(24, 20, seed)
    rect = (2, 2, 22, 18)
    lam = O.min_eig_map(img, rect)
    ref, A, _, Cc = library_min_eig(img, rect)
    assert np.max(np.abs(lam - ref) / np.maximum(A + Cc, 1.0)) < 1e-12


def test_constant_image_has_no_corners():
    xy, sc, nc = O.detect(np.full((120, 160), 90, np.uint8), 50)
    assert len(xy) == 0 and nc == 0


@pytest.mark.parametrize("axis", [0, 1])
def test_straight_edge_and_ramp_have_no_corners(axis):
    img = np.zeros((120, 160), np.uint8)
    if axis == 0:
        img[:, 80:] = 200
    else:
        img[60:, :] = 200
    assert len(O.detect(img, 50)[0]) == 0
    y, x = np.mgrid[0:120, 0:160]
    ramp = (x + y).astype(np.uint8)
    assert len(O.detect(ramp, 50)[0]) == 0


def test_bright_square_gives_its_four_corners():
    img = np.full((160, 200), 30, np.uint8)
    x0, y0, x1, y1 = 60, 50, 140, 110                       # square occupies [x0, x1) x [y0, y1)
    img[y0:y1, x0:x1] = 220
    xy, sc, _ = O.detect(img, 10, min_dist=10)
    assert len(xy) == 4
    geo = np.array([[x0 - 0.5, y0 - 0.5], [x1 - 0.5, y0 - 0.5], [x0 - 0.5, y1 - 0.5], [x1 - 0.5, y1 - 0.5]])
    for g in geo:
        d = np.min(np.hypot(*(xy - g).T))
        assert d <= 1.0
    assert np.all(np.diff(sc) <= 0)


def test_checkerboard_grid_intersections():
    cell = 16
    y, x = np.mgrid[0:160, 0:224]
    img = np.where(((x // cell) + (y // cell)) % 2 == 0, 40, 210).astype(np.uint8)
    xy, sc, _ = O.detect(img, 500, min_dist=10, roi=(16, 16))
    assert len(xy) > 0
    # every corner sits within 1 px of an intersection (multiples of 16, minus half a pixel)
    fx = np.abs(((xy[:, 0] + 0.5) / cell) - np.round((xy[:, 0] + 0.5) / cell)) * cell
    fy = np.abs(((xy[:, 1] + 0.5) / cell) - np.round((xy[:, 1] + 0.5) / cell)) * cell
    assert (fx <= 1.0).all() and (fy <= 1.0).all()
    # each crossing (at 16k - 1/2) with one of its two neighbouring pixels in the ROI is found once
    xs = [g for g in range(cell, 224, cell) if 16 <= g <= 224 - 16]
    ys = [g for g in range(cell, 160, cell) if 16 <= g <= 160 - 16]
    for gx in xs:
        for gy in ys:
            d = np.hypot(xy[:, 0] - (gx - 0.5), xy[:, 1] - (gy - 0.5))
            assert (d <= 1.0).sum() == 1
    assert len(xy) == len(xs) * len(ys)


def greedy_properties(order_xy, K, d, acc):
    """Defining properties of the greedy selection in order: (1) accepted points pairwise >= d;
    (2) every candidate processed before the K-th acceptance and not accepted conflicts with an
    earlier accepted one; (3) accepted candidates conflict with no earlier accepted one."""
    acc = list(acc)
    sacc = set(acc)
    last = acc[-1] if len(acc) == K else len(order_xy) - 1
    for a in acc:
        for b in acc:
            if a < b:
                assert np.sum((order_xy[a] - order_xy[b]) ** 2) >= d * d
    for i in range(last + 1):
        if i in sacc:
            continue
        assert any(np.sum((order_xy[i] - order_xy[a]) ** 2) < d * d for a in acc if a < i)


@settings(max_examples=60, deadline=None)
@given(seed=st.integers(0, 2**31 - 1), n=st.integers(0, 60), K=st.integers(1, 30), d=st.integers(1, 12))
def test_greedy_select_properties(seed, n, K, d):
    rng = np.random.default_rng(seed)
    xy = rng.integers(0, 40, size=(n, 2))
    acc = O.greedy_select(xy[:, 0], xy[:, 1], K, d)
    assert len(acc) <= K
    assert list(acc) == sorted(acc)
    if len(acc):
        greedy_properties(xy.astype(np.int64), K, d, acc)
    elif n:
        raise AssertionError("the first candidate is always accepted")


@pytest.mark.parametrize("seed", [5, 6])
def test_detect_order_threshold_spacing(seed):
    img = synth.smooth_random_image(200, 150, seed, sigma=2.0)
    K, q, d = 60, 0.01, 10
    xy, sc, nc = O.detect(img, K, q, d, roi=(16, 16))
    assert 0 < len(xy) <= K and nc >= len(xy)
    lam = O.min_eig_map(img, (16, 16, 184, 134))
    lmax = lam.max()
    assert sc[0] == lmax
    assert (sc >= q * lmax).all()
    # descending key, ties by (y, x)
    for a, b, pa, pb in zip(sc[:-1], sc[1:], xy[:-1], xy[1:]):
        assert a > b or (a == b and (pa[1], pa[0]) < (pb[1], pb[0]))
    # scores are the response at the reported pixel, every corner is a 3x3 local maximum
    for (x, y), s in zip(xy.astype(int), sc):
        assert lam[y - 16, x - 16] == s
        nb = lam[max(0, y - 17):y - 14, max(0, x - 17):x - 14]
        assert s >= nb.max()
    # inside the ROI, pairwise spacing
    assert (xy[:, 0] >= 16).all() and (xy[:, 0] < 184).all() and (xy[:, 1] >= 16).all() and (xy[:, 1] < 134).all()
    dd = np.sum((xy[:, None] - xy[None]) ** 2, -1) + np.eye(len(xy)) * 1e9
    assert dd.min() >= d * d
