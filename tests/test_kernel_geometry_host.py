"""Host-side checks of two index rules the kernels rely on for memory safety (no GPU).

* Photometric sums (an extension of Eq. 3 under the similarity of Eq. 7): a tile's source box is
  taken from the map of its four corner pixels, widened by one pixel, and staged when the map is
  far from degenerate (|a|, |b| < rho / 2) and the box fits 288 bytes x 80 rows. Every pixel's four
  bilinear taps must then lie inside the staged rows and columns. The map is evaluated here in the
  kernel's binary64 operation order (no fused operations), over many random maps and ragged tiles.
* Warp: wave w of a 256-thread workgroup takes the tile's columns 64 w .. 64 w + 63, its lanes 16
  per row and 4 rows at a time, each thread 4 consecutive pixels in 16 rows 4 apart. Every pixel of
  a 256 x 64 tile, clipped to the frame, is produced exactly once.
"""
import math

import numpy as np

TW, TH = 256, 32                   # photometric tile
SBW, SMAXR = 288, 79               # staged width (bytes) and rows of the next-frame box


def staged_box(t, X0, X1, Y0, Y1, cx, cy, rho):
    t0, t1, t2, t3 = t
    xs, ys = [], []
    for y in (Y0, Y1 - 1):
        for x in (X0, X1 - 1):
            dx, dy = (x - cx) / rho, (y - cy) / rho
            xs.append(((x + t0 * dx) - t1 * dy) + t2)
            ys.append(((y + t1 * dx) + t0 * dy) + t3)
    if not (abs(t0) < 0.5 * rho and abs(t1) < 0.5 * rho):
        return None
    a0 = (math.floor(min(xs)) - 1) & ~15
    by0 = math.floor(min(ys)) - 1
    nr = math.floor(max(ys)) + 2 - by0 + 1
    if not (math.floor(max(xs)) + 2 - a0 < SBW and nr <= SMAXR):
        return None
    return a0, by0, nr


def test_photometric_taps_inside_the_staged_box():
    rng = np.random.default_rng(11)
    checked = 0
    for case in range(400):
        w, h = int(rng.integers(40, 700)), int(rng.integers(30, 500))
        cx, cy, rho = (w - 1) / 2.0, (h - 1) / 2.0, max(w, h) / 2.0
        scale = [0.02, 0.1, 0.3, 0.49][case % 4]
        t = (rng.uniform(-scale, scale) * rho, rng.uniform(-scale, scale) * rho,
             rng.uniform(-40, 40), rng.uniform(-40, 40))
        ox0, oy0 = int(rng.integers(0, 20)), int(rng.integers(0, 20))
        ox1, oy1 = w - int(rng.integers(0, 20)), h - int(rng.integers(0, 20))
        if ox1 <= ox0 or oy1 <= oy0:
            continue
        tx = int(rng.integers(0, (ox1 - ox0 + TW - 1) // TW))
        ty = int(rng.integers(0, (oy1 - oy0 + TH - 1) // TH))
        X0, Y0 = ox0 + tx * TW, oy0 + ty * TH
        X1, Y1 = min(X0 + TW, ox1), min(Y0 + TH, oy1)
        box = staged_box(t, X0, X1, Y0, Y1, cx, cy, rho)
        if box is None:
            continue
        a0, by0, nr = box
        x = np.arange(X0, X1, dtype=np.float64)[None, :]
        y = np.arange(Y0, Y1, dtype=np.float64)[:, None]
        dx, dy = (x - cx) / rho, (y - cy) / rho
        px = ((x + t[0] * dx) - t[1] * dy) + t[2]
        py = ((y + t[1] * dx) + t[0] * dy) + t[3]
        col = np.floor(px).astype(np.int64) - a0
        row = np.floor(py).astype(np.int64) - by0
        assert col.min() >= 0 and col.max() + 1 <= SBW - 1, case
        assert row.min() >= 0 and row.max() + 1 <= nr - 1, case
        checked += 1
    assert checked > 200


def test_warp_lane_layout_covers_every_pixel_once():
    TWW, THW, WRPT = 256, 64, 16      # warp tile and rows per thread
    tid = np.arange(256)
    x4 = 64 * (tid >> 6) + 4 * (tid & 15)
    yq = (tid >> 4) & 3
    for W, H in [(256, 64), (100, 37), (333, 257), (64, 3), (5, 70)]:
        for oy in range(0, H, THW):
            for ox in range(0, W, TWW):
                hits = np.zeros((H, W), np.int64)
                for t in range(256):
                    xa = ox + x4[t]
                    nx = min(W - xa, 4)
                    yb = oy + yq[t]
                    ny = 0 if H - yb <= 0 else min((H - yb + 3) >> 2, WRPT)
                    for r in range(ny):
                        for q in range(max(nx, 0)):
                            hits[yb + 4 * r, xa + q] += 1
                tile = hits[oy:oy + THW, ox:ox + TWW]
                assert (tile == 1).all(), (W, H, ox, oy)
                assert hits.sum() == tile.size
