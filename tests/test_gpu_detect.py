"""GPU parity of detect_corners against the oracle (Section 3.1, Eq. 2): identical ordered corner
lists, bit-identical binary64 scores, identical counts."""
import numpy as np
import pytest
import torch

from helpers import dev, say
from oracle import oracle as O
from paper_1701_03572_amd import synth
from paper_1701_03572_amd import vstab as V

pytestmark = pytest.mark.gpu


def gpu_detect(imgs, K, q=0.01, d=10, roi=None, cap=None, istride=1, gate=None, gate_min=0, prefill=None):
    imgs = np.asarray(imgs)
    if imgs.ndim == 2:
        imgs = imgs[None]
    n, h, w = imgs.shape
    cap = cap or max(K, 1)
    mx, my = roi if roi is not None else O.roi_margins(w, h)
    p = V.vs_detect_params(K, q, d, mx, my)
    recs = n * istride
    xy = torch.full((recs, cap, 2), -7.0, dtype=torch.float32, device="cuda")
    sc = torch.full((recs, cap), -7.0, dtype=torch.float64, device="cuda")
    cnt = torch.full((recs,), -7, dtype=torch.int32, device="cuda")
    alive = torch.full((recs, cap), 9, dtype=torch.uint8, device="cuda")
    wsb = V.vs_detect_workspace(w, h, n)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    V.vs_detect_corners(dev(imgs), w * h, w, h, w, n, istride, None if gate is None else dev(np.asarray(gate, np.int32)),
                        gate_min, p, cap, xy, sc, cnt, alive, ws, wsb)
    torch.cuda.synchronize()
    return xy.cpu().numpy(), sc.cpu().numpy(), cnt.cpu().numpy(), alive.cpu().numpy()


def check_item(img, K, xy, sc, cnt, alive, q=0.01, d=10, roi=None):
    rxy, rsc, nc = O.detect(img, K, q, d, roi)
    assert cnt == len(rxy), (cnt, len(rxy), nc)
    np.testing.assert_array_equal(xy[:cnt], rxy.astype(np.float32))
    np.testing.assert_array_equal(sc[:cnt], rsc)                   # bit-identical binary64 keys
    assert (alive[:cnt] == 1).all() and (alive[cnt:] == 0).all()
    return nc


@pytest.mark.parametrize("name,K", [("tiny", 200), ("vga", 500), ("hd", 1000)])
def test_first_frames_of_each_workload(name, K):
    say("detect", name, K)
    seq = synth.make_sequence(name, n_frames=1)
    img = seq.frames[0]
    xy, sc, cnt, alive = gpu_detect(img, K)
    nc = check_item(img, K, xy[0], sc[0], cnt[0], alive[0])
    say("candidates", nc, "accepted", cnt[0])


@pytest.mark.parametrize("K,seed", [(1500, 0), (4000, 1), (1, 2), (37, 3)])
def test_noise_many_candidates(K, seed):
    # white noise has tens of thousands of local maxima: exercises the radix-select batches
    say("detect noise", K, seed)
    img = synth.random_image(640, 480, 100 + seed)
    xy, sc, cnt, alive = gpu_detect(img, K, cap=4096)
    nc = check_item(img, K, xy[0], sc[0], cnt[0], alive[0])
    assert nc > 4096


@pytest.mark.parametrize("w,h", [(33000, 24), (24, 33000)])
def test_frames_with_a_side_past_32768(w, h):
    # the selection decides distances in 64-bit arithmetic when a side exceeds 32768 (24-bit
    # products otherwise); a thin noise frame exercises that branch at a small size
    say("detect long frame", w, h)
    img = synth.random_image(w, h, 7)
    for d in (10, 40):
        xy, sc, cnt, alive = gpu_detect(img, 300, d=d, cap=300, roi=(2, 2))
        nc = check_item(img, 300, xy[0], sc[0], cnt[0], alive[0], d=d, roi=(2, 2))
        assert cnt[0] == 300 and nc > 300


def test_checkerboard_ties_and_spacing():
    say("detect checkerboard")
    y, x = np.mgrid[0:240, 0:320]
    img = np.where(((x // 8) + (y // 8)) % 2 == 0, 30, 220).astype(np.uint8)
    for d in (5, 10, 12):
        xy, sc, cnt, alive = gpu_detect(img, 3000, d=d, cap=3000)
        check_item(img, 3000, xy[0], sc[0], cnt[0], alive[0], d=d)


def test_flat_and_ramp_images_have_no_corners():
    y, x = np.mgrid[0:120, 0:160]
    for img in (np.full((120, 160), 80, np.uint8), (x + y).astype(np.uint8)):
        xy, sc, cnt, alive = gpu_detect(img, 50)
        assert cnt[0] == 0 and (alive == 0).all()


def test_quality_and_roi_variants():
    img = synth.smooth_random_image(400, 300, 8, sigma=2.0)
    for q, roi, d in [(0.0, (2, 2), 0), (0.2, (30, 10), 3), (0.9, (16, 16), 10)]:
        say("detect variant", q, roi, d)
        xy, sc, cnt, alive = gpu_detect(img, 700, q=q, d=d, roi=roi, cap=800)
        check_item(img, 700, xy[0], sc[0], cnt[0], alive[0], q=q, d=d, roi=roi)


def test_batch_istride_and_gate():
    seq = synth.make_sequence("tiny", n_frames=3)
    gate = np.full(9, 100, np.int32)
    gate[0], gate[6] = 3, 0                          # records 0 and 6 run, record 3 is gated off
    say("detect gate")
    xy, sc, cnt, alive = gpu_detect(seq.frames, 200, istride=3, gate=gate, gate_min=10)
    for i, rec in enumerate([0, 3, 6]):
        if rec == 3:
            assert cnt[rec] == -7 and (alive[rec] == 9).all() and (xy[rec] == -7).all()
        else:
            check_item(seq.frames[i], 200, xy[rec], sc[rec], cnt[rec], alive[rec])
    assert (cnt[[1, 2, 4, 5, 7, 8]] == -7).all()


def test_rejects_bad_arguments():
    img = synth.random_image(64, 48, 1)
    with pytest.raises(V.VsError):
        gpu_detect(img, 10, roi=(1, 1))
    with pytest.raises(V.VsError):
        gpu_detect(img, 10, cap=5)
    with pytest.raises(V.VsError):
        gpu_detect(img, 5000, cap=5000)
