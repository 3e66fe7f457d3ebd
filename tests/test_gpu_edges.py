"""Edge and size cases of the GPU path against the oracle.

* 3840x2160, the largest frames the serving workload carries: every pyramid level bit-exact,
  the 3000 strongest corners and their binary64 scores identical, a sample of 300 tracked points
  within the tracker's 0.01 px bar, and the warp within one level on at most 0.1 % of pixels.
* Small frames (48x40, two levels) through the whole sequence path: skip flags and model choices
  equal the oracle's, pair transforms within 0.02 px, stabilized pixels within one level.
* A batch of zero items is a no-op for every entry point: nothing is written.
"""
import numpy as np
import pytest
import torch

from helpers import dev, level_of, say
from oracle import oracle as O
from paper_1701_03572_amd import params, synth
from paper_1701_03572_amd import vstab as V
from paper_1701_03572_amd.pipeline import SequenceStabilizer
from test_gpu_detect import check_item, gpu_detect
from test_gpu_lk import compare

pytestmark = pytest.mark.gpu


def uhd_pair():
    sq = synth.make_sequence(synth.recipe("uhd", seed=5, motion="path"), n_frames=2)
    return sq.frames


def test_uhd_pyramid_corners_tracks_and_warp():
    f0, f1 = uhd_pair()
    h, w = f0.shape
    say("uhd pyramid", w, h)
    L = 5
    layout = V.vs_pyramid_layout(w, h, w, L)
    pyr = torch.zeros(layout.bytes, dtype=torch.uint8, device="cuda")
    V.vs_build_pyramid(dev(f0), w * h, pyr, layout.bytes, 1, layout)
    torch.cuda.synchronize()
    ref = O.pyramid(f0, L)
    for l in range(1, L):
        np.testing.assert_array_equal(level_of(pyr, layout, l), ref[l])

    say("uhd corners")
    K = 3000
    roi = O.roi_margins(w, h)
    xy, sc, cnt, alive = gpu_detect(f0, K, roi=roi)
    check_item(f0, K, xy[0], sc[0], cnt[0], alive[0], roi=roi)
    assert cnt[0] == K

    say("uhd tracks")
    pts = xy[0][:cnt[0]][:: cnt[0] // 300][:300].astype(np.float32)
    res = compare(f0, f1, pts, L)
    say(res)
    assert res["compared"] > 250

    say("uhd warp")
    a, b = 1.004 * np.cos(0.01), 1.004 * np.sin(0.01)
    cx, cy = (w - 1) / 2, (h - 1) / 2
    M = np.array([a, -b, cx - a * cx + b * cy + 3.25, b, a, cy - b * cx - a * cy - 1.5])
    out = torch.empty((h, w), dtype=torch.uint8, device="cuda")
    V.vs_warp_frame(dev(f0), w * h, w, h, w, dev(M), 6, out, w * h, w, 1, 0)
    torch.cuda.synchronize()
    d = np.abs(out.cpu().numpy().astype(int) - O.warp(f0, M).astype(int))
    assert d.max() <= 1 and (d > 0).mean() < 1e-3


def test_small_frames_whole_path():
    sq = synth.make_sequence("tiny", n_frames=12)
    frames = np.ascontiguousarray(sq.frames[:, 100:140, 130:178])     # 48 x 40
    n, h, w = frames.shape
    say("small frames", w, h)
    P = params.StabParams(levels=2, max_corners=30, min_dist=3, roi_mx=4, roi_my=4, win_half=3, min_valid=4,
                          radius=3, ransac_iters=16)
    ss = SequenceStabilizer(w, h, n, P)
    ss.run(dev(frames))
    torch.cuda.synchronize()
    got = ss.results(n)
    out = ss.out[:n].cpu().numpy()
    ref = O.stabilize(frames, P)
    cx, cy = (w - 1) / 2, (h - 1) / 2
    corners = np.array([[-cx, -cy], [cx, -cy], [-cx, cy], [cx, cy]])
    for p in range(n - 1):
        gi, ri = got["info"][p], ref["info"][p]
        assert gi["skipped"] == ri["skipped"], p
        tie = ri["decided_here"] and abs(ri["err_rigid"] - ri["err_sim"]) < 1e-6 * max(ri["err_sim"], 1e-30)
        if not tie:
            assert gi["model"] == ri["model"], p
        g, r = got["pair_params"][p], ref["pair_params"][p]
        ap = lambda t: np.stack([t[0] * corners[:, 0] - t[1] * corners[:, 1] + t[2],
                                 t[1] * corners[:, 0] + t[0] * corners[:, 1] + t[3]], 1)
        assert np.max(np.hypot(*(ap(g) - ap(r)).T)) < 0.02, p
    assert sum(not i["skipped"] for i in got["info"]) >= (n - 1) // 2
    d = np.abs(out.astype(int) - ref["warped"].astype(int))
    assert d.max() <= 1 and (d > 0).mean() < 1e-2


def test_zero_items_write_nothing():
    w, h, L, cap = 64, 48, 2, 8
    layout = V.vs_pyramid_layout(w, h, w, L)
    f = dev(synth.random_image(w, h, 3)[None])
    pyr = torch.full((layout.bytes,), 7, dtype=torch.uint8, device="cuda")
    V.vs_build_pyramid(f, w * h, pyr, layout.bytes, 0, layout)
    xy = torch.full((1, cap, 2), -3.0, dtype=torch.float32, device="cuda")
    sc = torch.full((1, cap), -3.0, dtype=torch.float64, device="cuda")
    cnt = torch.full((1,), -3, dtype=torch.int32, device="cuda")
    al = torch.full((1, cap), 5, dtype=torch.uint8, device="cuda")
    ws = torch.empty(256, dtype=torch.uint8, device="cuda")
    V.vs_detect_corners(f, w * h, w, h, w, 0, 1, None, 0, V.vs_detect_params(cap, 0.01, 3, 4, 4), cap, xy, sc, cnt, al,
                        ws, 0)
    st = torch.full((1, cap), 5, dtype=torch.uint8, device="cuda")
    V.vs_track_lk(f, pyr, f, pyr, 0, 0, 0, 1, layout, xy, al, cap, V.vs_lk_params(3, 10, 1e-3, 1e-2, 1, 1.0), xy, st)
    fst = torch.zeros(V.FIT_STATE_BYTES, dtype=torch.uint8, device="cuda")
    V.vs_fit_state_init(fst)
    torch.cuda.synchronize()
    before = fst.clone()
    prm = torch.full((1, 4), -3.0, dtype=torch.float64, device="cuda")
    m6 = torch.full((1, 6), -3.0, dtype=torch.float64, device="cuda")
    info = torch.full((V.FIT_INFO_BYTES,), 5, dtype=torch.uint8, device="cuda")
    fp = V.vs_fit_params(V.VS_HYBRID3, 8, 1.0, 1, 0, 3, 20, (w - 1) / 2, (h - 1) / 2)
    V.vs_fit_motion(xy, xy, al, cap, 0, fp, 0, fst, prm, m6, info, st, ws, 0)
    out = torch.full((1, h, w), 9, dtype=torch.uint8, device="cuda")
    mats = torch.zeros((1, 6), dtype=torch.float64, device="cuda")
    V.vs_warp_frame(f, w * h, w, h, w, mats, 6, out, w * h, w, 0, 0)
    torch.cuda.synchronize()
    assert (pyr == 7).all() and (xy == -3).all() and (sc == -3).all() and (cnt == -3).all() and (al == 5).all()
    assert (st == 5).all() and (prm == -3).all() and (m6 == -3).all() and (info == 5).all() and (out == 9).all()
    assert torch.equal(fst, before)
