"""The per-frame driver's ready event (vs_stream.ready_event): recorded by every push once the
frames it emits are written, before the re-detection that serves only the next pair.

A side stream that waits only for each push's ready event copies the emitted frames; the copies
must equal the outputs of a run without events (after a full synchronisation). The run covers
re-detection frames (every 5th) and the causal smoother, which emits every frame in its own push.
"""
import pytest
import torch

from helpers import say
from paper_1701_03572_amd import params, synth
from paper_1701_03572_amd.pipeline import Stabilizer

pytestmark = pytest.mark.gpu


def test_outputs_complete_at_the_ready_event():
    sq = synth.make_sequence("tiny", n_frames=16, device="cuda")
    frames = sq.frames.contiguous()
    n, h, w = frames.shape
    say("ready event", w, h, n)
    P = params.PRESETS["tiny"].replace(smooth_mode=params.SMOOTH_CAUSAL)
    ref = Stabilizer(w, h, P, out_slots=n)
    for j in range(n):
        ref.push(frames[j])
    torch.cuda.synchronize()
    expect = ref.out[:n].clone()

    st = Stabilizer(w, h, P, out_slots=n)
    side = torch.cuda.Stream()
    copies = {}
    for j in range(n):
        ev = torch.cuda.Event()
        emitted = st.push(frames[j], ready=ev)
        assert [e for e, _ in emitted] == [j]
        side.wait_event(ev)
        with torch.cuda.stream(side):
            copies[j] = emitted[0][1].clone()
    torch.cuda.synchronize()
    for j in range(n):
        assert torch.equal(copies[j], expect[j]), j
    assert torch.equal(st.out[:n], expect)
