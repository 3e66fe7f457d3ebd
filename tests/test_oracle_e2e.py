"""End-to-end oracle runs on seeded synthetic sequences whose pair transforms are known exactly
(each frame is the previous one moved by a known similarity), following the paper's
motion-estimation workflow (Section 4.1) and motion compensation (Section 5.1)."""
import numpy as np

from oracle import oracle as O
from paper_1701_03572_amd import params, synth


def transform_error_px(p_est, p_gt, w, h):
    """max over the frame's corners and centre of |T_est(x) - T_gt(x)| (centred coordinates)."""
    cx, cy = (w - 1) / 2, (h - 1) / 2
    pts = np.array([[-cx, -cy], [cx, -cy], [-cx, cy], [cx, cy], [0, 0]])

    def ap(p):
        a, b, tx, ty = p
        return np.stack([a * pts[:, 0] - b * pts[:, 1] + tx, b * pts[:, 0] + a * pts[:, 1] + ty], 1)

    return np.max(np.hypot(*(ap(p_est) - ap(p_gt)).T))


def test_tiny_sequence_recovers_ground_truth():
    seq = synth.make_sequence("tiny", n_frames=12)
    P = params.PRESETS["tiny"].replace(model=params.SIMILARITY)
    out = O.stabilize(seq.frames, P)
    gt = seq.pair_params_centred()
    errs = [transform_error_px(a, b, 320, 240) for a, b in zip(out["pair_params"], gt)]
    assert max(errs) < 0.05
    assert np.median(errs) < 0.02
    assert out["detect_frames"] == [0, 5, 10]
    assert all(not i["skipped"] for i in out["info"])
    # stabilised output keeps the frame size, warps every frame
    assert out["warped"].shape == seq.frames.shape


def test_blank_frames_skip_and_redetect():
    seq = synth.make_sequence("tiny", n_frames=8)
    frames = seq.frames.copy()
    frames[3] = 100                                     # a flat frame: nothing to track
    P = params.PRESETS["tiny"]
    out = O.stabilize(frames, P, warp_frames=False)
    info = out["info"]
    assert info[2]["skipped"] == 1                      # 2 -> 3 lands on the blank frame
    assert info[3]["skipped"] == 1                      # 3 -> 4 starts from no corners
    np.testing.assert_array_equal(out["pair_params"][2], [1, 0, 0, 0])
    assert 3 in out["detect_frames"] and 4 in out["detect_frames"]
    assert not info[4]["skipped"]
    assert np.isfinite(out["mats"]).all()
