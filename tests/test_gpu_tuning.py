"""Launch tuning never changes a result: pyramids, corners, tracks (positions, statuses, round-trip
errors, valid counts, work counters), warps and fits (parameters, 2x3 models, records, inlier flags,
dwell state) are bit-identical under every per-XCD mapping choice, 1, 2 or 4 points per tracking
workgroup (a capacity that is not a multiple of the group size included), any corner-response
segment height and any number of fit workgroups in flight. The autotuner times the candidates, installs the fastest and caches it."""
import numpy as np
import pytest
import torch

from helpers import dev, say
from paper_1701_03572_amd import synth
from paper_1701_03572_amd import tuning as T
from paper_1701_03572_amd import vstab as V

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def defaults():
    T.set_tuning(None)
    yield
    T.set_tuning(None)


def run_all(frames, K=501, L=4):
    n, h, w = frames.shape
    fs = h * w
    layout = V.vs_pyramid_layout(w, h, w, L)
    ps = layout.bytes
    pyr = torch.zeros((n, ps), dtype=torch.uint8, device="cuda")
    V.vs_build_pyramid(frames, fs, pyr, ps, n, layout)
    seg = (n - 1) // 5
    dp = V.vs_detect_params(K, 0.01, 10, 32, 24)
    xy = torch.zeros((n, K, 2), dtype=torch.float32, device="cuda")
    al = torch.zeros((n, K), dtype=torch.uint8, device="cuda")
    cnt = torch.zeros(n, dtype=torch.int32, device="cuda")
    wsb = V.vs_detect_workspace(w, h, seg)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    V.vs_detect_corners(frames, 5 * fs, w, h, w, seg, 5, None, 0, dp, K, xy, None, cnt, al, ws, wsb)
    lkp = V.vs_lk_params(10, 30, 1e-3, 1e-2, 1, 1.0)
    dst = torch.zeros((n, K, 2), dtype=torch.float32, device="cuda")
    st = torch.zeros((n, K), dtype=torch.uint8, device="cuda")
    fe = torch.zeros((n, K), dtype=torch.float32, device="cuda")
    nv = torch.zeros(n, dtype=torch.int32, device="cuda")
    wk = torch.zeros(2 * seg, dtype=torch.int64, device="cuda")
    f0, p0 = frames.data_ptr(), pyr.data_ptr()
    V.vs_track_lk(f0, p0, f0 + fs, p0 + ps, 5 * fs, 5 * ps, seg, 5, layout, xy, al, K, lkp, dst, st, fe, nv, None, None,
                  wk)
    th = torch.linspace(-0.02, 0.02, n, dtype=torch.float64, device="cuda")
    cx, cy = (w - 1) / 2, (h - 1) / 2
    a, b = torch.cos(th), torch.sin(th)
    mats = torch.stack([a, -b, cx - a * cx + b * cy + 2.5, b, a, cy - b * cx - a * cy - 1.25], 1).contiguous()
    out = torch.empty_like(frames)
    V.vs_warp_frame(frames, fs, w, h, w, mats, 6, out, fs, w, n, 0)
    # the fit of the tracked pairs (every 5th record) as consecutive items
    src5, dst5, st5 = (t[0::5][:seg].contiguous() for t in (xy, dst, st))
    fp = V.vs_fit_params(V.VS_HYBRID3, 128, 1.0, 5, 1, 10, 2, cx, cy)
    fstate = torch.zeros(V.FIT_STATE_BYTES, dtype=torch.uint8, device="cuda")
    V.vs_fit_state_init(fstate)
    prm = torch.zeros((seg, 4), dtype=torch.float64, device="cuda")
    m6 = torch.zeros((seg, 6), dtype=torch.float64, device="cuda")
    info = torch.zeros(seg * V.FIT_INFO_BYTES, dtype=torch.uint8, device="cuda")
    inl = torch.zeros((seg, K), dtype=torch.uint8, device="cuda")
    fwsb = V.vs_fit_workspace(seg, K)
    fws = torch.empty(fwsb, dtype=torch.uint8, device="cuda")
    V.vs_fit_motion(src5, dst5, st5, K, seg, fp, 0, fstate, prm, m6, info, inl, fws, fwsb)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in (pyr, xy, cnt, dst, st, fe, nv, wk, out, prm, m6, info, inl, fstate)]


@pytest.mark.parametrize("t", [T.Tuning(1, 1, 1, 1), T.Tuning(65536, 65536, 65536, 2), T.Tuning(8, 8, 8, 4),
                               T.Tuning(1, 65536, 8, 4), T.Tuning(det_rows=12, fit_groups=64),
                               T.Tuning(det_rows=240, fit_groups=16384), T.Tuning(det_rows=37, fit_groups=100)])
def test_results_do_not_depend_on_the_tuning(t):
    frames = dev(synth.make_sequence("vga", n_frames=46).frames)      # 9 items: above and below the thresholds
    ref = run_all(frames)
    say("tuning", t)
    T.set_tuning(t)
    got = run_all(frames)
    for r, g in zip(ref, got):
        np.testing.assert_array_equal(g, r)
    assert ref[6][::5].sum() > 0


def test_autotune_installs_and_caches(tmp_path):
    path = str(tmp_path / "tuning.json")
    frames = dev(synth.make_sequence("vga", n_frames=21).frames)
    t, timings = T.autotune(frames, 300, 4, reps=2, path=path)
    say("autotuned", t, {k: min(v.values()) for k, v in timings.items()})
    assert T.get_tuning() == t
    assert set(timings) == {"pyramid", "lk", "warp", "detect", "fit"} and len(timings["lk"]) == 9
    T.set_tuning(None)
    assert T.apply(640, 480, 300, path) == t and T.get_tuning() == t
