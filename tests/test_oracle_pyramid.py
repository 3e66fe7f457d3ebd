"""Pins of the oracle's Gaussian pyramid (Section 3.2: image pyramids for large motion).

Each pin checks the oracle against something other than itself: scipy's correlation with the
binomial kernel built from math.comb, closed forms for constant and linear images, the impulse
response, and shift equivariance.
"""
import math

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st
from scipy import ndimage

from oracle import oracle as O

BINOM = np.array([math.comb(4, k) for k in range(5)], dtype=np.float64)   # Pascal row 4


def scipy_level(img: np.ndarray) -> np.ndarray:
    """Binomial 5x5 correlation with scipy ('mirror' = reflect without repeating the edge),
    even-sample decimation, one round half up."""
    k2 = np.outer(BINOM, BINOM)
    full = ndimage.correlate(img.astype(np.float64), k2, mode="mirror")
    dec = full[0::2, 0::2]
    return np.floor(dec / 256.0 + 0.5).astype(np.uint8)


@settings(max_examples=40, deadline=None)
@given(w=st.integers(3, 41), h=st.integers(3, 37), seed=st.integers(0, 2**31 - 1))
def test_matches_scipy_correlation(w, h, seed):
    img = np.random.default_rng(seed).integers(0, 256, size=(h, w), dtype=np.uint8)
    got = O.pyr_down(img)
    assert got.shape == ((h + 1) // 2, (w + 1) // 2)
    np.testing.assert_array_equal(got, scipy_level(img))


@pytest.mark.parametrize("w,h", [(320, 240), (641, 479), (1920, 1080)])
def test_large_sizes_match_scipy(w, h):
    img = np.random.default_rng(w * h).integers(0, 256, size=(h, w), dtype=np.uint8)
    np.testing.assert_array_equal(O.pyr_down(img), scipy_level(img))


def test_level_sizes_ceil_halving():
    pyr = O.pyramid(np.zeros((1080, 1920), np.uint8), 5)
    assert [p.shape for p in pyr] == [(1080, 1920), (540, 960), (270, 480), (135, 240), (68, 120)]


@pytest.mark.parametrize("v", [0, 1, 77, 128, 255])
def test_constant_image_stays_constant(v):
    pyr = O.pyramid(np.full((97, 131), v, np.uint8), 4)
    for p in pyr:
        assert (p == v).all()


def test_linear_ramp_preserved_in_interior():
    # the binomial kernel has unit sum and zero first moment: linear images pass unchanged
    h, w = 64, 96
    y, x = np.mgrid[0:h, 0:w]
    img = (x + 2 * y).astype(np.uint8)             # max 95 + 126 = 221
    lv = O.pyr_down(img)
    yy, xx = np.mgrid[0:lv.shape[0], 0:lv.shape[1]]
    inner = (slice(1, -1), slice(1, -1))
    np.testing.assert_array_equal(lv[inner], (2 * xx + 4 * yy)[inner].astype(np.uint8))


@pytest.mark.parametrize("px,py", [(20, 30), (21, 30), (20, 31), (21, 31)])
def test_impulse_response_is_binomial(px, py):
    # a pixel of 256 is spread by the polyphase components of C(4, k): even sites see taps
    # (1, 6, 1), odd sites (4, 4).
    img = np.zeros((64, 64), np.uint16)
    img[py, px] = 255
    lv = O.pyr_down(img.astype(np.uint8)).astype(np.float64)
    expect = np.zeros_like(lv)
    for yo in range(lv.shape[0]):
        for xo in range(lv.shape[1]):
            i, j = px - 2 * xo, py - 2 * yo
            if abs(i) <= 2 and abs(j) <= 2:
                expect[yo, xo] = math.floor(255 * BINOM[i + 2] * BINOM[j + 2] / 256.0 + 0.5)
    np.testing.assert_array_equal(lv, expect)


def test_shift_equivariance_multi_level():
    big = np.random.default_rng(3).integers(0, 256, size=(200, 260), dtype=np.uint8)
    t = 8                                          # 2^3: level l shifts by t / 2^l
    a = O.pyramid(big[40:168, 40:232], 4)
    b = O.pyramid(big[40 - t:168 - t, 40 - t:232 - t], 4)
    for l in range(4):
        s = t >> l
        m = 8                                      # stay clear of border-affected samples
        np.testing.assert_array_equal(a[l][m:-m - s, m:-m - s], b[l][m + s:-m, m + s:-m])
