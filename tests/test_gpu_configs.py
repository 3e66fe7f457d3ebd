"""Parity at the workloads' full sizes, in the launch configuration the benchmark times (the
segment-parallel sequence path over every frame of the workload).

Stage by stage, each oracle stage is fed the GPU path's own inputs to that stage, so every output
is compared with what the paper's method computes from the same data:
* corners (Section 3.1, Eq. 2) on every detection frame: identical ordered lists;
* tracking (Section 3.2, Eqs. 3-6, backward check of Section 4.1) of every pair (sampled segments at
  1080p): the tracker bar (0.01 px, decision-boundary exemptions at most 1 %);
* the fit (Section 4, Eq. 7, hybrid and skip rule of Section 4.1) of every pair from the GPU's tracks,
  the hybrid state carried in pair order: identical inlier sets, counts, skips and model choices,
  parameters within 1e-8;
* smoothing (Sections 5.1, 6) of the GPU's pair parameters: every matrix within 1e-9;
* the warp (Section 5) of every frame (sampled frames at 1080p) under the GPU's matrix: within one
  grey level.
End to end, against the oracle run on its own binary64 tracks (the tiny and VGA workloads): the same
detections, skips and model choices (ties within 1e-12 relative excepted), pair transforms within
0.01 px over the frame.
"""
import concurrent.futures as cf

import numpy as np
import pytest
import torch

from helpers import dev, lk_parity, say, transform_err
from oracle import oracle as O
from paper_1701_03572_amd import params, synth
from paper_1701_03572_amd.pipeline import SequenceStabilizer

pytestmark = pytest.mark.gpu

WORKERS = 16


def _run_gpu(frames_dev, P):
    n, h, w = frames_dev.shape
    ss = SequenceStabilizer(w, h, n, P)
    ss.run(frames_dev)
    torch.cuda.synchronize()
    res = ss.results(n)
    res["out"] = ss.out[:n].cpu().numpy()
    return res


def _roi(P, w, h):
    return P.roi(w, h)


def check_detections(frames, res, P, frames_idx):
    w, h = frames.shape[2], frames.shape[1]
    with cf.ThreadPoolExecutor(WORKERS) as ex:
        refs = list(ex.map(lambda f: O.detect(frames[f], P.max_corners, P.quality, P.min_dist, _roi(P, w, h))[0],
                           frames_idx))
    for f, rxy in zip(frames_idx, refs):
        cnt = int(res["alive_src"][f].sum())
        assert cnt == len(rxy), (f, cnt, len(rxy))
        np.testing.assert_array_equal(res["src"][f][:cnt], rxy.astype(np.float32))
        assert not res["alive_src"][f][cnt:].any()
    return len(frames_idx)


def check_tracks(frames, res, P, pairs):
    n, h, w = frames.shape
    lkp = dict(win_half=P.win_half, max_iter=P.max_iter, eps=P.eps, min_eig=P.min_eig, fb=P.fb,
               fb_thresh=P.fb_thresh)

    def one(p):
        al = res["alive_src"][p]
        ref = O.track_lk(O.pyramid(frames[p], P.levels), O.pyramid(frames[p + 1], P.levels),
                         res["src"][p].astype(np.float64), al, with_margin=True, **lkp)
        return lk_parity(res["dst"][p], res["status"][p], ref, w, h, al, **lkp)

    with cf.ThreadPoolExecutor(WORKERS) as ex:
        reps = list(ex.map(one, pairs))
    tot = {k: sum(r[k] for r in reps) for k in ("n", "compared", "excluded", "status_mismatch", "capped_beyond_tol")}
    tot["max_err"] = max(r["max_err"] for r in reps)
    tot["pairs"] = len(pairs)
    say("tracks", tot)
    assert tot["excluded"] <= 0.01 * tot["n"]
    return tot


def check_fits(res, P, w, h):
    fp = O.fit_params(P.model, P.ransac_iters, P.inlier_thresh, P.seed, P.stream_id, P.min_valid, P.dwell, w, h)
    st = O.new_hybrid_state()
    worst = 0.0
    n_pairs = len(res["pair_params"])
    for p in range(n_pairs):
        prm, m6, info, inl = O.fit_pair_affine(res["src"][p].astype(np.float64), res["dst"][p].astype(np.float64),
                                               res["status"][p], fp, p, st)
        gi = res["info"][p]
        for k in ("skipped", "model", "decided_here", "n_valid", "n_inliers"):
            assert gi[k] == info[k], (p, k, gi[k], info[k])
        np.testing.assert_array_equal(res["inliers"][p][:len(inl)], inl, err_msg="pair %d" % p)
        d = np.abs(res["pair_params"][p] - prm) / np.maximum(1.0, np.abs(prm))
        worst = max(worst, float(d.max()))
    say("fits: %d pairs, worst parameter difference %.2e" % (n_pairs, worst))
    assert worst <= 1e-8
    return worst


def check_smoothing(res, P, w, h):
    n = len(res["mats"])
    _, _, mats = O.smooth(res["pair_params"], n, P.smooth_mode, P.radius, P.kalman_ratio, P.crop, w, h)
    d = float(np.max(np.abs(res["mats"] - mats) / np.maximum(1.0, np.abs(mats))))
    say("smoothing: %d matrices, worst difference %.2e" % (n, d))
    assert d <= 1e-9
    return d


def check_warps(frames, res, P, idx):
    with cf.ThreadPoolExecutor(WORKERS) as ex:
        refs = list(ex.map(lambda j: O.warp(frames[j], res["mats"][j], P.border), idx))
    off = 0
    for j, r in zip(idx, refs):
        d = np.abs(res["out"][j].astype(int) - r.astype(int))
        assert d.max() <= 1, (j, int(d.max()))
        off += int((d > 0).sum())
    say("warps: %d frames, %d pixels differ by one level (%.2e)" % (len(idx), off, off / (len(idx) * frames[0].size)))


def check_end_to_end(frames, res, P):
    n, h, w = frames.shape
    ref = O.stabilize(frames, P, warp_frames=False, workers=WORKERS)
    for f in ref["detect_frames"]:
        if f < n - 1:
            cnt = int(res["alive_src"][f].sum())
            np.testing.assert_array_equal(res["src"][f][:cnt], ref["detections"][f].astype(np.float32))
    errs, ties = [], 0
    for p in range(n - 1):
        gi, ri = res["info"][p], ref["info"][p]
        assert gi["skipped"] == ri["skipped"], p
        assert gi["decided_here"] == ri["decided_here"], p
        tie = ri["decided_here"] and abs(ri["err_rigid"] - ri["err_sim"]) < 1e-12 * ri["err_sim"]
        ties += int(tie)
        if not tie:
            assert gi["model"] == ri["model"], p
        errs.append(transform_err(res["pair_params"][p], ref["pair_params"][p], w, h))
    errs = np.array(errs)
    say("end to end: %d pairs, transform difference max %.2e px, median %.2e px, ties %d" % (
        n - 1, errs.max(), np.median(errs), ties))
    assert errs.max() < 0.01
    return ref


@pytest.mark.parametrize("name", ["tiny", "vga"])
def test_whole_workload(name):
    rec = synth.RECIPES[name]
    P = params.PRESETS[name]
    say("whole workload", name, rec.n_frames)
    sq = synth.make_sequence(name)
    frames = sq.frames
    n, h, w = frames.shape
    res = _run_gpu(dev(frames), P)
    det = sorted({f for f in range(0, n - 1, P.redetect_every)} |
                 {p + 1 for p in range(n - 2) if res["info"][p]["skipped"]})
    check_detections(frames, res, P, det)
    check_tracks(frames, res, P, list(range(n - 1)))
    check_fits(res, P, w, h)
    check_smoothing(res, P, w, h)
    check_warps(frames, res, P, list(range(n)))
    check_end_to_end(frames, res, P)


def test_hd_workload_stage_by_stage():
    rec = synth.RECIPES["hd"]
    P = params.PRESETS["hd"]
    n = rec.n_frames
    say("hd workload", n)
    sq = synth.make_sequence("hd", device="cuda")
    res = _run_gpu(sq.frames, P)
    frames = sq.frames.cpu().numpy()
    w, h = rec.width, rec.height
    skipped = [p for p in range(n - 1) if res["info"][p]["skipped"]]
    assert not skipped
    check_detections(frames, res, P, list(range(0, n - 1, P.redetect_every)))
    segs = list(range(0, 120, 11)) + [119]
    check_tracks(frames, res, P, [5 * m + s for m in segs for s in range(5) if 5 * m + s < n - 1])
    check_fits(res, P, w, h)
    check_smoothing(res, P, w, h)
    check_warps(frames, res, P, list(range(0, n, 25)) + [n - 1])
