"""Error bound of the corner response's FP32 score estimate (host emulation, no GPU).

The response kernel keeps a pixel, drops it, or flags it for an exact comparison by comparing FP32
estimates of the Shi-Tomasi score 2 det / (tr + sqrt(disc)) within a relative band of 1e-5; the
result is the exact set of 3x3 maxima only if every estimate is within half the band of the exact
score. The estimate takes the box-summed Sobel tensor (A, B, C), integers below 2^24 in magnitude,
and forms det with Kahan's compensated 2x2 determinant, disc = (A - C)^2 + 4 fl(B^2) with one fused
rounding, the sum A + C, a square root and a reciprocal of at most one ulp error, and the product.

Here every float32 operation is emulated exactly: products and sums of these integers are exact in
binary64, so a fused multiply-add is the binary64 value rounded once to float32. The square root
and the reciprocal are pushed by a full ulp in the direction that hurts most. The estimate must stay
within 10 * 2^-24 of the exact score (computed with rational arithmetic), and its sign test must
agree with det > 0, on random tensors and on tensors built to make det cancel.
"""
from fractions import Fraction
import math

import numpy as np

U = 2.0 ** -24
F32 = np.float32


def f32(x) -> float:
    return float(F32(x))


def ulp_push(x: float, up: bool) -> float:
    return float(np.nextafter(F32(x), F32(np.inf) if up else F32(-np.inf)))


def estimate(A: int, B: int, C: int, sq_up: bool, rcp_up: bool) -> float:
    a, b, c = float(A), float(B), float(C)       # exact in float32 (|.| < 2^24)
    w = f32(b * b)
    e = f32(w - b * b)                           # fma(-b, b, w): exact in binary64, one rounding
    det = f32(f32(a * c - w) + e)                # fma(a, c, -w), then the compensated sum
    if not det > 0.0:
        return 0.0
    dm = f32(a - c)
    disc = f32(dm * dm + 4.0 * w)                # fma(dm, dm, 4 w)
    sf = ulp_push(f32(math.sqrt(disc)), sq_up)   # a square root within one ulp
    den = f32(f32(a + c) + sf)
    r = ulp_push(f32(1.0 / den), rcp_up)         # a reciprocal within one ulp
    return f32(f32(2.0 * det) * r)


def exact_score(A: int, B: int, C: int) -> float:
    det = A * C - B * B
    if det <= 0:
        return 0.0
    disc = (A - C) ** 2 + 4 * B * B
    root = Fraction(0)
    if disc:
        # Newton steps from the binary64 root: far below float32 precision after three
        root = Fraction(math.sqrt(disc))
        for _ in range(3):
            root = (root + Fraction(disc) / root) / 2
    return float(Fraction(2 * det) / (A + C + root))


def check(A: int, B: int, C: int):
    ex = exact_score(A, B, C)
    for sq_up in (False, True):
        for rcp_up in (False, True):
            est = estimate(A, B, C, sq_up, rcp_up)
            assert (est > 0.0) == (A * C - B * B > 0), (A, B, C)
            if ex > 0.0:
                assert abs(est - ex) <= 10 * U * ex, (A, B, C, est, ex, abs(est - ex) / ex / U)


def test_random_tensors():
    rng = np.random.default_rng(11)
    lim = 9 * 1020 * 1020          # 3x3 box of squared Sobel responses of 8-bit images
    for _ in range(4000):
        A = int(rng.integers(0, lim))
        C = int(rng.integers(0, lim))
        bm = int(math.isqrt(A * C)) if A * C > 0 else 1
        B = int(rng.integers(-bm, bm + 1))
        check(A, B, C)


def test_cancelling_determinants():
    rng = np.random.default_rng(12)
    lim = 9 * 1020 * 1020
    for _ in range(4000):
        A = int(rng.integers(1, lim))
        C = int(rng.integers(1, lim))
        B = math.isqrt(A * C) - int(rng.integers(0, 3))   # det = A C - B^2 tiny against A C
        for b in (B, -B):
            check(A, b, C)


def test_degenerate_tensors():
    for A, B, C in [(0, 0, 0), (5, 0, 0), (0, 0, 7), (4, 2, 1), (4, -2, 1), (9, 3, 1), (1, 0, 1), (16777215, 0, 1),
                    (16777215, 16777214, 16777215), (16777215, -16777214, 16777215)]:
        check(A, B, C)
