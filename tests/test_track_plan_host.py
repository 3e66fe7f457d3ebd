"""The launch plan of the segment-parallel tracking (host logic, no GPU).

``pipeline.track_segments`` must issue, for a sequence of n frames in 5-frame segments:
one vs_track_lk_segments call over every segment from pair 0 (no gate), then for s = 1 .. 4 a
re-detection of frame s and a re-tracking from pair s, both gated on the valid count of pair
s - 1 of each segment and both over the segments that have pair s; the last segment's pair count
when it is short; and, with ``per_pair=True``, one vs_track_lk call per pair with its chained
outputs and gated re-detection. The binding's calls are replaced by recorders, so only the plan is
checked; the GPU tests check that both plans give the same records bit for bit.
"""
import types

import pytest

from paper_1701_03572_amd import params, pipeline
from paper_1701_03572_amd import vstab as V


class FakeTensor:
    def __init__(self, addr, shape):
        self.addr, self.shape = addr, shape

    def data_ptr(self):
        return self.addr


def records(cap, n):
    o = types.SimpleNamespace()
    o.src = FakeTensor(0x10000000, (n, cap, 2))
    o.asrc = FakeTensor(0x20000000, (n, cap))
    o.dst = FakeTensor(0x30000000, (n, cap, 2))
    o.status = FakeTensor(0x40000000, (n, cap))
    o.fb_err = FakeTensor(0x50000000, (n, cap))
    o.n_valid = FakeTensor(0x60000000, (n,))
    o.count = FakeTensor(0x70000000, (n,))
    o.score = FakeTensor(0x80000000, (n, cap))
    o.det_ws, o.det_ws_bytes = FakeTensor(0x90000000, (1,)), 1
    return o


def run_plan(monkeypatch, n_frames, per_pair):
    calls = []
    monkeypatch.setattr(V, "vs_track_lk_segments", lambda *a, **k: calls.append(("seg", a)))
    monkeypatch.setattr(V, "vs_track_lk", lambda *a, **k: calls.append(("pair", a)))
    monkeypatch.setattr(V, "vs_detect_corners", lambda *a, **k: calls.append(("det", a)))
    P = params.PRESETS["hd"]
    e, cap = P.redetect_every, P.max_corners
    n_pairs = n_frames - 1
    o = records(cap, n_frames)
    fs, ps = 1920 * 1080, 2_800_000
    pipeline.track_segments(o, 0x1000, 0x2000, fs, ps,
                            lambda s: (n_pairs - 1 - s) // e + 1 if 0 <= s <= n_pairs - 1 else 0, P, "layout",
                            "lkp", "dp", 1920, 1080, per_pair=per_pair)
    return calls, P, o, fs, ps


@pytest.mark.parametrize("n_frames", [600, 601, 598, 6, 3])
def test_segment_plan(monkeypatch, n_frames):
    calls, P, o, fs, ps = run_plan(monkeypatch, n_frames, per_pair=False)
    e, cap = P.redetect_every, P.max_corners
    n_pairs = n_frames - 1
    n_seg = -(-n_pairs // e)
    last = n_pairs - (n_seg - 1) * e                    # pairs of the last segment
    nv = o.n_valid.data_ptr()
    kind = [c[0] for c in calls]
    assert "pair" not in kind
    # the first call: every segment from pair 0, no gate
    seg = [c[1] for c in calls if c[0] == "seg"]
    first = seg[0]
    assert first[:11] == (0x1000, 0x2000, e * fs, e * ps, fs, ps, n_seg, e, e, last, 0)
    assert first[20] is None                            # gate
    # then, for each later pair s present: a gated re-detection of frame s, then a gated re-tracking
    expect = []
    for s in range(1, e):
        n_s = (n_pairs - 1 - s) // e + 1 if s <= n_pairs - 1 else 0
        if n_s <= 0:
            break
        expect += [("det", s, n_s), ("seg", s, n_s)]
    got = []
    for k, a in calls[1:]:
        if k == "det":
            s = (a[0] - 0x1000) // fs
            assert a[0] == 0x1000 + s * fs and a[6] == e and a[8] == P.min_valid
            assert a[7] == nv + (s - 1) * 4            # gate: valid count of pair s - 1
            assert a[11] == o.src.data_ptr() + s * cap * 2 * 4
            got.append(("det", s, a[5]))
        else:
            s = a[10]
            assert a[20] == nv + (s - 1) * 4 and a[21] == P.min_valid
            assert a[9] == (last if a[6] == n_seg else e)
            got.append(("seg", s, a[6]))
    assert got == expect


@pytest.mark.parametrize("n_frames", [600, 13])
def test_per_pair_plan(monkeypatch, n_frames):
    calls, P, o, fs, ps = run_plan(monkeypatch, n_frames, per_pair=True)
    e, cap = P.redetect_every, P.max_corners
    n_pairs = n_frames - 1
    pairs = [a for k, a in calls if k == "pair"]
    dets = [a for k, a in calls if k == "det"]
    assert len(pairs) == min(e, n_pairs)
    for s, a in enumerate(pairs):
        assert a[0] == 0x1000 + s * fs and a[2] == 0x1000 + (s + 1) * fs
        assert a[6] == (n_pairs - 1 - s) // e + 1
        chained = s < e - 1
        assert (a[17] is not None) == chained and (a[18] is not None) == chained
    # a gated re-detection of frame s + 1 after every pair s that has a successor in its segment
    def pairs_of(s):
        return (n_pairs - 1 - s) // e + 1 if 0 <= s <= n_pairs - 1 else 0
    assert [(a[0] - 0x1000) // fs for a in dets] == [s + 1 for s in range(len(pairs)) if s < e - 1 and pairs_of(s + 1) > 0]
    assert all(a[7] == o.n_valid.data_ptr() + ((a[0] - 0x1000) // fs - 1) * 4 for a in dets)
