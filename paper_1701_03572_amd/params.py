"""Parameter presets of the stabilization path (plain constants, no arithmetic).

Constants the paper fixes: corner budget 50 (Section 3.1), re-detection every 5 frames
(Section 3.2), hybrid dwell of 20 frames (Section 4.1), smoothing radius 10 in the real-time
version (Section 6). Everything else is a reading of a silent paper, chosen per workload.
"""
from __future__ import annotations

import dataclasses

RIGID, SIMILARITY, HYBRID, AFFINE, HYBRID3 = 0, 1, 2, 3, 4
SMOOTH_CENTERED, SMOOTH_CAUSAL, SMOOTH_KALMAN = 0, 1, 2


@dataclasses.dataclass(frozen=True)
class StabParams:
    levels: int = 3
    max_corners: int = 50
    quality: float = 0.01
    min_dist: int = 10
    roi_mx: int | None = None      # None: max(16, W // 20)
    roi_my: int | None = None      # None: max(16, H // 20)
    redetect_every: int = 5
    win_half: int = 10             # 21 x 21 window
    max_iter: int = 30
    eps: float = 1e-3              # px, stop when |eta| < eps
    min_eig: float = 1e-2          # lambda_min(G) / window size
    fb: bool = True
    fb_thresh: float = 1.0         # px
    model: int = HYBRID
    ransac_iters: int = 128
    inlier_thresh: float = 1.0     # px
    seed: int = 1701
    stream_id: int = 0
    min_valid: int = 10
    dwell: int = 20
    smooth_mode: int = SMOOTH_CENTERED
    radius: int = 15
    kalman_ratio: float = 0.02
    crop: float = 0.0
    border: int = 0
    photometric_steps: int = 0     # Gauss-Newton photometric refinement of each fitted pair (0: off)
    photometric_margin: int | None = None   # None: max(16, min(W, H) // 10)

    def roi(self, w: int, h: int) -> tuple[int, int]:
        mx = self.roi_mx if self.roi_mx is not None else max(16, w // 20)
        my = self.roi_my if self.roi_my is not None else max(16, h // 20)
        return mx, my

    def photo_margin(self, w: int, h: int) -> int:
        return self.photometric_margin if self.photometric_margin is not None else max(16, min(w, h) // 10)

    def replace(self, **kw) -> "StabParams":
        return dataclasses.replace(self, **kw)


PRESETS = {
    # 320x240, 3 levels, 200 corners, 21x21 window, 30 iterations, moving average radius 15
    "tiny": StabParams(levels=3, max_corners=200, radius=15, smooth_mode=SMOOTH_CENTERED),
    # 640x480, 4 levels, 500 corners, robust fit (1 px), Kalman smoothing
    "vga": StabParams(levels=4, max_corners=500, smooth_mode=SMOOTH_KALMAN, seed=1702),
    # 1920x1080, 5 levels, 1000 corners, robust fit, hybrid, moving average radius 15
    "hd": StabParams(levels=5, max_corners=1000, radius=15, smooth_mode=SMOOTH_CENTERED, seed=1703),
    # the paper's own budget: 50 corners, radius 10
    "paper": StabParams(levels=4, max_corners=50, radius=10, smooth_mode=SMOOTH_CENTERED),
}
