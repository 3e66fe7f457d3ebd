"""Serving with continuous batching (Section 6's real-time version across streams): the frames of all
admitted streams of a class are processed together in ticks.

* A stream's outputs do not depend on what else is served: alone, and in a mix where other streams of
  its class share its ticks and streams of other classes run beside them, bit for bit; and they equal
  the stream pushed alone through the per-frame path.
* Served streams against the oracle (a subsample): stabilized frames within one grey level almost
  everywhere (the oracle tracks in binary64; the per-stage parity of the same kernels is tested
  elsewhere).
* Admission checks the HBM budget before allocating; streams that do not fit wait with their frames
  buffered, every frame of every stream is emitted, finished streams' buffers are reused by later
  streams of their class, and the reserved memory returns to 0 once idle buffers are released.
* A short paced replay of Poisson arrivals reports latencies and throughput.
"""
import numpy as np
import pytest
import torch

from helpers import dev, say
from oracle import oracle as O
from paper_1701_03572_amd import synth
from paper_1701_03572_amd.params import SMOOTH_CAUSAL, StabParams
from paper_1701_03572_amd.pipeline import Stabilizer, member_bytes
from paper_1701_03572_amd.serve import ServedStream, StreamServer, poisson_workload, simulate

pytestmark = pytest.mark.gpu

GB = 1 << 30


def host_clip(name, n, seed):
    r = synth.recipe(name, seed=seed, motion="path")
    f = synth.make_sequence(r, n_frames=n).frames
    t = torch.empty(f.shape, dtype=torch.uint8, pin_memory=True)
    t.copy_(torch.from_numpy(f))
    return t


def collect():
    outs = {}

    def on_emit(sid, e, view):
        outs[(sid, e)] = view.clone()           # on the class's queue, ordered after the warp
    return outs, on_emit


def serve(server, streams, ticks_between=1):
    """streams: [(sid, clip, P, start tick)]; one frame per stream per tick from its start."""
    outs, on_emit = collect()
    n_ticks = max(st + clip.shape[0] for _, clip, _, st in streams)
    for t in range(n_ticks):
        for sid, clip, P, st in streams:
            if t == st:
                server.open(sid, clip.shape[2], clip.shape[1], P)
            if st <= t < st + clip.shape[0]:
                server.submit(sid, clip[t - st])
                if t == st + clip.shape[0] - 1:
                    server.close(sid)
        server.tick(on_emit=on_emit)
    server.drain(on_emit=on_emit)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in outs.items()}


def test_stream_alone_equals_stream_in_a_mix():
    a = host_clip("tiny", 16, 41)
    b = host_clip("vga", 9, 42)
    c = host_clip("tiny", 11, 43)
    d = host_clip("tiny", 13, 44)
    PA = StabParams(levels=3, max_corners=200, smooth_mode=SMOOTH_CAUSAL, stream_id=7, seed=70)
    PB = StabParams(levels=4, max_corners=500, smooth_mode=SMOOTH_CAUSAL, stream_id=8, seed=80)
    PC = StabParams(levels=3, max_corners=100, smooth_mode=SMOOTH_CAUSAL, stream_id=9, seed=90)
    PD = StabParams(levels=3, max_corners=300, smooth_mode=SMOOTH_CAUSAL, stream_id=10, seed=100)
    alone = serve(StreamServer(8 * GB, capacity=500), [(1, a, PA, 0)])
    mixed = serve(StreamServer(8 * GB, capacity=500), [(2, c, PC, 0), (1, a, PA, 2), (3, b, PB, 1), (4, d, PD, 5)])
    assert sorted(e for s, e in alone) == list(range(16))
    for e in range(16):
        np.testing.assert_array_equal(alone[(1, e)], mixed[(1, e)])
    # the per-frame path pushed alone, with the same capacity, gives the same outputs
    st = Stabilizer(320, 240, PA, out_slots=16, capacity=500)
    fr = dev(a.numpy())
    for j in range(16):
        st.push(fr[j])
    st.flush()
    torch.cuda.synchronize()
    ref = st.out.cpu().numpy()
    for e in range(16):
        np.testing.assert_array_equal(alone[(1, e)], ref[e])
    # every frame of every stream of the mix was emitted
    for sid, n in ((1, 16), (2, 11), (3, 9), (4, 13)):
        assert sorted(e for s, e in mixed if s == sid) == list(range(n))


def test_served_streams_match_the_oracle():
    clips = [host_clip("tiny", 18, 61), host_clip("tiny", 15, 62), host_clip("vga", 12, 63)]
    Ps = [StabParams(levels=3, max_corners=200, smooth_mode=SMOOTH_CAUSAL, stream_id=1, seed=11),
          StabParams(levels=3, max_corners=150, smooth_mode=SMOOTH_CAUSAL, stream_id=2, seed=12),
          StabParams(levels=4, max_corners=400, smooth_mode=SMOOTH_CAUSAL, stream_id=3, seed=13)]
    got = serve(StreamServer(8 * GB, capacity=500), [(k, c, P, k) for k, (c, P) in enumerate(zip(clips, Ps))])
    for k in (0, 2):                              # the subsample checked against the oracle
        ref = O.stabilize(clips[k].numpy(), Ps[k])
        n = clips[k].shape[0]
        d = np.abs(np.stack([got[(k, e)] for e in range(n)]).astype(int) - ref["warped"].astype(int))
        say("served stream", k, "pixels off by more than one level:", int((d > 1).sum()), "of", d.size)
        assert (d > 1).mean() < 1e-3


def test_admission_by_budget_buffers_frames_and_releases_memory():
    P = StabParams(levels=3, max_corners=200, smooth_mode=SMOOTH_CAUSAL)
    one = member_bytes(320, 240, P, 200, 2, 2)
    probe = StreamServer(64 * GB, capacity=200, max_concurrent=4)
    before = torch.cuda.memory_allocated()
    assert probe.open(0, 320, 240, P)
    cls_bytes = probe.used - one
    assert torch.cuda.memory_allocated() - before <= probe.used    # the reservation covers what was allocated
    probe.close(0)
    probe.drain()
    assert probe.used > 0 and len(probe.classes[next(iter(probe.classes))].pool) == 1   # buffers pooled
    probe.release_idle()
    assert probe.used == 0 and not probe.classes
    budget = cls_bytes + int(2.5 * one)                              # room for two streams at a time
    clips = [host_clip("tiny", 6 + k, 70 + k) for k in range(4)]
    server = StreamServer(budget, capacity=200, max_concurrent=4)
    outs, on_emit = collect()
    for k, c in enumerate(clips):
        server.open(k, 320, 240, P.replace(stream_id=k))
    assert sorted(server.streams) == [0, 1] and [m.sid for m in server.waiting] == [2, 3]
    assert server.used <= server.budget
    for k, c in enumerate(clips):
        for j in range(c.shape[0]):
            server.submit(k, c[j])                                   # queued streams buffer their frames
        server.close(k)
    while server.has_work():
        server.tick(on_emit=on_emit)
        assert server.used <= server.budget and len(server.streams) <= 2
    torch.cuda.synchronize()
    assert not server.streams and not server.waiting
    assert server.used == cls_bytes + 2 * one          # two streams' buffers pooled, reused by the later two
    server.release_idle()
    assert server.used == 0 and not server.classes
    for k, c in enumerate(clips):
        assert sorted(e for s, e in outs if s == k) == list(range(c.shape[0]))
    with pytest.raises(RuntimeError):
        tiny = StreamServer(one // 2, capacity=200)
        tiny.open(9, 320, 240, P)
        tiny.submit(9, clips[0][0])
        tiny.close(9)
        simulate(tiny, [], clips, paced=False)


def test_paced_poisson_replay():
    pools = [host_clip("tiny", 24, 51), host_clip("vga", 24, 52)]
    classes = [(320, 240, 3, 0), (640, 480, 4, 1)]
    wl = poisson_workload(1.0, 6.0, (0.2, 0.6), 30.0, classes, (100, 400), seed=3, warm_start_s=0.3)
    assert len(wl) >= 2 and all(isinstance(s, ServedStream) for s in wl)
    res = simulate(StreamServer(16 * GB, capacity=400), wl, pools, paced=True)
    say(res)
    assert res["frames_out"] == res["frames_in"] == sum(s.n_frames for s in wl)
    assert 0 < res["latency_ms_p50"] <= res["latency_ms_p99"] < 1000
    sat = simulate(StreamServer(16 * GB, capacity=400), wl, pools, paced=False)
    say(sat)
    assert sat["frames_out"] == res["frames_out"] and sat["frames_per_s"] > 0 and sat["latency_ms_p99"] is None
    assert sat["mean_items_per_push"] > 1


def test_prepared_classes_and_pooled_buffers_give_the_same_outputs():
    """A stream served on reused (pooled) buffers of an earlier stream equals the stream served on
    fresh buffers, bit for bit."""
    a = host_clip("tiny", 9, 81)
    b = host_clip("tiny", 7, 82)
    PA = StabParams(levels=3, max_corners=200, smooth_mode=SMOOTH_CAUSAL, stream_id=1, seed=5)
    PB = StabParams(levels=3, max_corners=120, smooth_mode=SMOOTH_CAUSAL, stream_id=2, seed=6)
    fresh = serve(StreamServer(8 * GB, capacity=200), [(2, b, PB, 0)])
    server = StreamServer(8 * GB, capacity=200)
    assert server.prepare(320, 240, PA, streams=1)
    reused = serve(server, [(1, a, PA, 0), (2, b, PB, 9)])      # b starts after a ended: a's buffers
    for e in range(7):
        np.testing.assert_array_equal(fresh[(2, e)], reused[(2, e)])
