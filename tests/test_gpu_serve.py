"""Serving loop: a stream's outputs do not depend on what else is served (alone vs in a mix, bit for
bit), admission queues streams that do not fit the HBM budget and admits them when memory is
released, and a short paced replay of Poisson arrivals reports latencies and throughput."""
import numpy as np
import pytest
import torch

from helpers import say
from paper_1701_03572_amd import synth
from paper_1701_03572_amd.params import SMOOTH_CAUSAL, StabParams
from paper_1701_03572_amd.serve import StreamServer, poisson_workload, simulate

pytestmark = pytest.mark.gpu

GB = 1 << 30


def host_clip(name, n, seed):
    r = synth.recipe(name, seed=seed, motion="path")
    f = synth.make_sequence(r, n_frames=n).frames
    t = torch.empty(f.shape, dtype=torch.uint8, pin_memory=True)
    t.copy_(torch.from_numpy(f))
    return t


def serve_stream(server, sid, clip, P, others=()):
    """Push ``clip`` through stream ``sid``, interleaving one frame of every other (sid, clip, P)
    after each frame; returns host copies of sid's outputs in order. Outputs are copied on the
    stream's own queue (ordered after the warp that wrote them, before a later push reuses the slot)."""
    h, w = clip.shape[1:]
    assert server.open(sid, w, h, P)
    for osid, oclip, oP in others:
        assert server.open(osid, oclip.shape[2], oclip.shape[1], oP)
    q = server.streams[sid].queue
    outs = {}
    for j in range(clip.shape[0]):
        for e, t in server.submit(sid, clip[j]):
            with torch.cuda.stream(q):
                outs[e] = t.clone()
        for osid, oclip, oP in others:
            server.submit(osid, oclip[j % oclip.shape[0]])
    for e, t in server.close(sid):
        with torch.cuda.stream(q):
            outs[e] = t.clone()
    for osid, _, _ in others:
        server.close(osid)
    torch.cuda.synchronize()
    return [outs[e].cpu().numpy() for e in sorted(outs)]


def test_stream_alone_equals_stream_in_a_mix():
    a = host_clip("tiny", 16, 41)
    b = host_clip("vga", 9, 42)
    c = host_clip("tiny", 11, 43)
    PA = StabParams(levels=3, max_corners=200, smooth_mode=SMOOTH_CAUSAL, stream_id=7)
    PB = StabParams(levels=4, max_corners=500, smooth_mode=SMOOTH_CAUSAL, stream_id=8)
    PC = StabParams(levels=3, max_corners=100, smooth_mode=SMOOTH_CAUSAL, stream_id=9)
    alone = serve_stream(StreamServer(4 * GB, queues=1), 1, a, PA)
    mixed = serve_stream(StreamServer(4 * GB, queues=3), 1, a, PA, others=[(2, b, PB), (3, c, PC)])
    assert len(alone) == len(mixed) == 16
    for x, y in zip(alone, mixed):
        np.testing.assert_array_equal(x, y)


def test_admission_queues_and_releases():
    P = StabParams(levels=3, max_corners=200, smooth_mode=SMOOTH_CAUSAL)
    probe = StreamServer(64 * GB)
    assert probe.open(0, 320, 240, P)
    one = probe.streams[0].reserved
    probe.close(0)
    server = StreamServer(int(2.5 * one))
    assert server.open(1, 320, 240, P) and server.open(2, 320, 240, P)
    assert not server.open(3, 320, 240, P)
    assert 3 not in server.streams and len(server.waiting) == 1
    server.close(1)
    assert 3 in server.streams and not server.waiting
    assert server.used <= server.budget


def test_paced_poisson_replay():
    pools = [host_clip("tiny", 24, 51), host_clip("vga", 24, 52)]
    classes = [(320, 240, 3, 0), (640, 480, 4, 1)]
    wl = poisson_workload(1.0, 6.0, (0.2, 0.6), 30.0, classes, (100, 400), seed=3)
    assert len(wl) >= 2
    res = simulate(StreamServer(16 * GB), wl, pools, paced=True)
    say(res)
    assert res["admitted"] == len(wl)
    assert res["frames_out"] == sum(s.n_frames for s in wl)
    assert 0 < res["latency_ms_p50"] <= res["latency_ms_p99"] < 1000
    sat = simulate(StreamServer(16 * GB), wl, pools, paced=False)
    say(sat)
    assert sat["frames_out"] == res["frames_out"] and sat["frames_per_s"] > 0 and sat["latency_ms_p99"] is None
