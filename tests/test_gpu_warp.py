"""GPU parity of warp_frame against the oracle (Section 5 image composition): exact on the pinned
special cases, within one grey level elsewhere."""
import math

import numpy as np
import pytest
import torch

from helpers import dev, say
from oracle import oracle as O
from paper_1701_03572_amd import synth
from paper_1701_03572_amd import vstab as V

pytestmark = pytest.mark.gpu


def gpu_warp(img, M, border=0):
    h, w = img.shape
    out = torch.empty((h, w), dtype=torch.uint8, device="cuda")
    V.vs_warp_frame(dev(img), 0, w, h, w, dev(np.asarray(M, np.float64).reshape(6)), 6, out, 0, w, 1, border)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("M", [[1, 0, 0, 0, 1, 0], [1, 0, 3, 0, 1, -5], [1, 0, -17, 0, 1, 8],
                               [-1, 0, 319, 0, -1, 239], [1, 0, -0.5, 0, 1, 0], [1, 0, 0, 0, 1, 0.5]])
def test_exact_cases(M):
    say("warp exact", M)
    img = synth.random_image(320, 240, 5)
    np.testing.assert_array_equal(gpu_warp(img, M), O.warp(img, M))


@pytest.mark.parametrize("w,h,seed", [(320, 240, 0), (641, 479, 1), (1920, 1080, 2), (37, 23, 3)])
def test_similarity_within_one_level(w, h, seed):
    say("warp similarity", w, h, seed)
    rng = np.random.default_rng(seed)
    img = synth.smooth_random_image(w, h, seed, sigma=1.3)
    th, s = rng.normal(0, 0.05), 1 + rng.normal(0, 0.03)
    a, b = s * math.cos(th), s * math.sin(th)
    M = [a, -b, rng.normal(0, 10), b, a, rng.normal(0, 10)]
    for border in (0, 200):
        g, o = gpu_warp(img, M, border).astype(int), O.warp(img, M, border).astype(int)
        d = np.abs(g - o)
        assert d.max() <= 1
        assert (d > 0).mean() < 1e-3


def test_batch_of_frames_and_matrices():
    n, w, h = 4, 320, 240
    say("warp batch", n)
    seq = synth.make_sequence("tiny", n_frames=n)
    rng = np.random.default_rng(9)
    mats = np.array([[1 + rng.normal(0, 0.01), rng.normal(0, 0.02), rng.normal(0, 4), rng.normal(0, 0.02),
                      1 + rng.normal(0, 0.01), rng.normal(0, 4)] for _ in range(n)])
    out = torch.zeros((n, h, w), dtype=torch.uint8, device="cuda")
    V.vs_warp_frame(dev(seq.frames), w * h, w, h, w, dev(mats), 6, out, w * h, w, n, 0)
    torch.cuda.synchronize()
    for i in range(n):
        d = np.abs(out[i].cpu().numpy().astype(int) - O.warp(seq.frames[i], mats[i]).astype(int))
        assert d.max() <= 1


def test_degenerate_matrix_gives_border():
    img = synth.random_image(64, 48, 1)
    out = gpu_warp(img, [1e-30, 0, 0, 0, 1e-30, 0], border=9)
    assert (out.ravel()[1:] == 9).all()            # only the origin maps inside the source
    out = gpu_warp(img, [float("nan")] * 6, border=7)
    assert (out == 7).all()


@pytest.mark.parametrize("theta,scale", [(0.087, 1.0), (0.5, 1.0), (0.0, 0.5), (-0.03, 1.04)])
def test_rotation_and_zoom_both_paths(theta, scale):
    """Moderate rotations stage the tile's source box in LDS; strong rotation or zoom-out give boxes
    too large for it and take the direct per-pixel path. Both must match the oracle, borders included."""
    say("warp rotation/zoom", theta, scale)
    w, h = 640, 480
    img = synth.smooth_random_image(w, h, 11, sigma=1.3)
    a, b = scale * math.cos(theta), scale * math.sin(theta)
    cx, cy = w / 2, h / 2
    M = [a, -b, cx - a * cx + b * cy + 3.25, b, a, cy - b * cx - a * cy - 2.5]
    for border in (0, 131):
        g, o = gpu_warp(img, M, border).astype(int), O.warp(img, M, border).astype(int)
        d = np.abs(g - o)
        assert d.max() <= 1
        assert (d > 0).mean() < 1e-3
