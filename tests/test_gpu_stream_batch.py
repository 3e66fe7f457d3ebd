"""The batched per-frame step (vs_batch_push): many streams advanced one frame each per call, one
launch per stage for all of them (the real-time version of Section 6 across streams).

* Every stream's outputs in a batch equal the same stream pushed alone through vs_stream_push, bit for
  bit: streams of different corner budgets, seeds, lengths and start times, joining and leaving
  between steps, with skipped pairs (blank frames), under each smoothing mode.
* One batched stream against the oracle (Sections 3-5): skips and model choices equal, pair
  transforms within 0.01 px, stabilized frames within one grey level of the oracle's warp under the
  same matrices.
* A captured step replayed frame after frame equals the eager steps.
* Streams of another class, unattached or repeated slots are rejected before any work is enqueued.
"""
import numpy as np
import pytest
import torch

from helpers import dev, say, transform_err
from oracle import oracle as O
from paper_1701_03572_amd import params, synth
from paper_1701_03572_amd import vstab as V
from paper_1701_03572_amd.pipeline import Stabilizer, StreamBatch

pytestmark = pytest.mark.gpu

W, H = 320, 240


def stream_frames(k, n, blank=()):
    r = synth.recipe("tiny", seed=4100 + k, motion="path")
    f = synth.make_sequence(r, n_frames=n).frames.copy()
    for b in blank:
        f[b] = 90
    return dev(f)


def run_alone(frames, P, cap):
    n = frames.shape[0]
    st = Stabilizer(W, H, P, out_slots=n, capacity=cap)
    outs, hist = {}, []
    for j in range(n):
        for e, t in st.push(frames[j]):
            outs[e] = t
        if j > 0:
            hist.append((st.pair_params.clone(), st.info.clone()))
    for e, t in st.flush():
        outs[e] = t
    torch.cuda.synchronize()
    return {e: t.cpu().numpy() for e, t in outs.items()}, hist


def run_batched(streams, P_class, cap, ticks):
    """streams: list of (frames, P, start step); returns per stream ({frame: output}, pair history)."""
    sb = StreamBatch(W, H, P_class, cap, max_streams=8, detect_chunk=3)
    members, slots = {}, {}
    outs = [dict() for _ in streams]
    hist = [[] for _ in streams]
    for t in range(ticks):
        for k, (fr, P, start) in enumerate(streams):
            if t == start:
                st = sb.member(P, out_slots=fr.shape[0], ring=fr)
                slots[k] = sb.attach(st)
                members[k] = st
        active = [k for k, (fr, P, start) in enumerate(streams) if k in slots and start <= t < start + fr.shape[0]]
        if not active:
            continue
        res = sb.push([slots[k] for k in active])
        for k in active:
            for e, o in res[slots[k]]:
                outs[k][e] = o
            if t > streams[k][2]:
                st = members[k]
                hist[k].append((st.pair_params.clone(), st.info.clone()))
        for k in active:
            fr, P, start = streams[k]
            if t == start + fr.shape[0] - 1:          # the stream's last frame: leave and flush
                st = sb.detach(slots.pop(k))
                for e, o in st.flush():
                    outs[k][e] = o
    torch.cuda.synchronize()
    return [{e: t.cpu().numpy() for e, t in o.items()} for o in outs], hist


@pytest.mark.parametrize("mode", [params.SMOOTH_CENTERED, params.SMOOTH_CAUSAL, params.SMOOTH_KALMAN])
def test_batched_streams_equal_streams_alone(mode):
    base = params.PRESETS["tiny"].replace(smooth_mode=mode)
    cap = 200
    spec = [(0, 22, 0, 200, ()), (1, 17, 3, 150, (6,)), (2, 17, 7, 80, ()), (3, 19, 2, 200, (4, 12))]
    streams = []
    for k, n, start, K, blank in spec:
        P = base.replace(max_corners=K, seed=900 + k, stream_id=k)
        streams.append((stream_frames(k, n, blank), P, start))
    say("batched vs alone, smoothing mode", mode)
    got, ghist = run_batched(streams, base.replace(max_corners=cap), cap, 30)
    for k, (fr, P, start) in enumerate(streams):
        ref, rhist = run_alone(fr, P, cap)
        n = fr.shape[0]
        assert sorted(got[k]) == list(range(n)) == sorted(ref)
        for e in range(n):
            np.testing.assert_array_equal(got[k][e], ref[e], err_msg="stream %d frame %d" % (k, e))
        assert len(ghist[k]) == len(rhist) == n - 1
        for (gp, gi), (rp, ri) in zip(ghist[k], rhist):
            assert torch.equal(gp, rp) and torch.equal(gi, ri)
    skipped = [V.fit_info_to_dicts(i)[0]["skipped"] for _, i in ghist[3]]
    assert skipped[3] and skipped[4]            # the blank frame 4 forces two skipped pairs


def test_batched_stream_matches_the_oracle():
    P = params.PRESETS["tiny"].replace(max_corners=150, seed=77, stream_id=5, smooth_mode=params.SMOOTH_CAUSAL)
    frames = [stream_frames(10, 26), stream_frames(11, 20, (9,)), stream_frames(12, 24)]
    streams = [(frames[0], P, 0), (frames[1], P.replace(max_corners=200, seed=78, stream_id=6), 1),
               (frames[2], P.replace(max_corners=100, seed=79, stream_id=7), 4)]
    got, ghist = run_batched(streams, P.replace(max_corners=200), 200, 30)
    for k in (0, 1):
        fr = frames[k].cpu().numpy()
        Pk = streams[k][1]
        ref = O.stabilize(fr, Pk)
        n = fr.shape[0]
        errs = []
        for p in range(n - 1):
            gp = ghist[k][p][0].cpu().numpy()[0]
            gi = V.fit_info_to_dicts(ghist[k][p][1])[0]
            ri = ref["info"][p]
            assert gi["skipped"] == ri["skipped"] and gi["decided_here"] == ri["decided_here"], (k, p)
            tie = ri["decided_here"] and abs(ri["err_rigid"] - ri["err_sim"]) < 1e-12 * ri["err_sim"]
            if not tie:
                assert gi["model"] == ri["model"], (k, p)
            errs.append(transform_err(gp, ref["pair_params"][p], W, H))
        say("stream", k, "max transform difference", max(errs))
        assert max(errs) < 0.01
        d = np.abs(np.stack([got[k][e] for e in range(n)]).astype(int) - ref["warped"].astype(int))
        assert (d > 1).mean() < 1e-3


def test_graph_replay_equals_eager_steps():
    P = params.PRESETS["tiny"].replace(smooth_mode=params.SMOOTH_KALMAN)
    frames = [stream_frames(20 + k, 12) for k in range(3)]      # Kalman: no lag, rings of 2+ frames
    Ks = (200, 120, 60)

    def build():
        sb = StreamBatch(W, H, P, 200, max_streams=4, detect_chunk=4)
        slots = [sb.attach(sb.member(P.replace(max_corners=K, stream_id=k, seed=k), out_slots=12, ring=fr))
                 for k, (fr, K) in enumerate(zip(frames, Ks))]
        return sb, slots

    sb, slots = build()
    for _ in range(12):
        sb.push(slots)
    torch.cuda.synchronize()
    eager = [sb.members[s].out.cpu().numpy() for s in slots]

    sb2, slots2 = build()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        sb2.push(slots2)
    for _ in range(12):
        g.replay()
        torch.cuda.synchronize()             # the program's own work between replays
        _ = sb2.members[slots2[0]].pair_params.sum().item()
    sb2.note_replayed(slots2, 11)
    torch.cuda.synchronize()
    for s, e in zip(slots2, eager):
        st = sb2.members[s]
        assert st._s.next_frame == 12 and st._s.emitted == 12
        np.testing.assert_array_equal(st.out.cpu().numpy(), e)


def test_rejected_arguments_enqueue_nothing():
    P = params.PRESETS["tiny"]
    sb = StreamBatch(W, H, P, 200, max_streams=2, detect_chunk=1)
    fr = stream_frames(30, 17)
    s0 = sb.attach(sb.member(P, ring=fr))
    with pytest.raises(V.VsError):
        sb.attach(Stabilizer(W, H, P.replace(min_valid=5), capacity=200, ring=fr))     # another class
    with pytest.raises(V.VsError):
        sb.attach(Stabilizer(W, H, P, capacity=100, ring=fr))                         # another capacity
    with pytest.raises(V.VsError):
        V.vs_batch_push(sb.b, [s0, s0])                                                # listed twice
    with pytest.raises(V.VsError):
        V.vs_batch_push(sb.b, [1])                                                     # not attached
    with pytest.raises(V.VsError):
        StreamBatch(W, H, P.replace(photometric_steps=2), 200, max_streams=2)
    torch.cuda.synchronize()
    assert sb.members[s0]._s.next_frame == 0
