"""Heterogeneous batching of independent streams (several resolutions, corner budgets and pyramid
depths in one batch): every stream's results equal the same stream processed alone, bit for bit;
a captured HIP graph replayed several times (with eager work and synchronisations in between)
reproduces the eager results every time."""
import numpy as np
import pytest
import torch

from helpers import say
from paper_1701_03572_amd import params, synth
from paper_1701_03572_amd.batch import MultiStabilizer, StreamSpec
from paper_1701_03572_amd.pipeline import SequenceStabilizer

pytestmark = pytest.mark.gpu


def mixed(n_streams, n_frames, base_seed):
    specs, frames = [], []
    for s, (r, k, levels) in enumerate(synth.mixed_streams(n_streams, n_frames, base_seed)):
        P = params.PRESETS["vga"].replace(levels=levels, max_corners=k, stream_id=s, seed=1705)
        seq = synth.make_sequence(r, n_frames=n_frames, device="cuda")
        specs.append(StreamSpec(r.width, r.height, n_frames, P))
        frames.append(seq.frames.contiguous())
    return specs, frames


def same_info(a, b):
    """Fit info records equal field by field (NaN equals NaN: pairs without a model decision)."""
    if len(a) != len(b):
        return False
    for x, y in zip(a, b):
        for k in x:
            u, v = x[k], y[k]
            if not (u == v or (isinstance(u, float) and isinstance(v, float) and np.isnan(u) and np.isnan(v))):
                return False
    return True


def alone(spec, frames):
    ss = SequenceStabilizer(spec.width, spec.height, spec.n_frames, spec.params)
    ss.run(frames)
    torch.cuda.synchronize()
    return ss.results(spec.n_frames), ss.out[:spec.n_frames].clone()


def test_mixed_batch_equals_streams_alone():
    specs, frames = mixed(7, 13, base_seed=1705)
    say("streams", [(s.width, s.height, s.params.max_corners, s.params.levels) for s in specs])
    ms = MultiStabilizer(specs)
    assert len(ms.classes) >= 2
    for i, f in enumerate(frames):
        ms.load(i, f)
    ms.run()
    torch.cuda.synchronize()
    for i, spec in enumerate(specs):
        ref, ref_out = alone(spec, frames[i])
        got = ms.results(i)
        np.testing.assert_array_equal(got["pair_params"], ref["pair_params"])
        assert same_info(got["info"], ref["info"])
        np.testing.assert_array_equal(got["mats"], ref["mats"])
        np.testing.assert_array_equal(got["n_valid"], ref["n_valid"])
        assert torch.equal(ms.output(i), ref_out)


def test_graph_replays_reproduce_eager_results():
    specs, frames = mixed(4, 11, base_seed=1706)
    ms = MultiStabilizer(specs)
    for i, f in enumerate(frames):
        ms.load(i, f)
    ms.run()
    torch.cuda.synchronize()
    eager = [(ms.results(i), ms.output(i).clone()) for i in range(len(specs))]
    ms.capture_graph()
    for rep in range(3):
        # eager work of the program between replays: clobber the outputs, then replay
        for c in ms.classes:
            c.out.zero_()
            c.pair_params.zero_()
        torch.cuda.synchronize()
        ms.replay()
        torch.cuda.synchronize()
        for i in range(len(specs)):
            got = ms.results(i)
            np.testing.assert_array_equal(got["pair_params"], eager[i][0]["pair_params"])
            np.testing.assert_array_equal(got["mats"], eager[i][0]["mats"])
            assert torch.equal(ms.output(i), eager[i][1]), (rep, i)


def test_frame_step_batch_equals_sequence_batch_eager_and_replayed():
    """The per-frame-step batch (each step: the next frame of every stream, one launch set per class)
    gives every stream the outputs of the whole-sequence batch, bit for bit; so do replays of one
    captured step, and a second pass after a reset."""
    from paper_1701_03572_amd.batch import FrameStepBatch
    specs, frames = mixed(6, 12, base_seed=1707)
    ms = MultiStabilizer(specs)
    for i, f in enumerate(frames):
        ms.load(i, f)
    ms.run()
    torch.cuda.synchronize()
    ref = [ms.output(i).clone() for i in range(len(specs))]
    fb = FrameStepBatch(specs, frames, detect_chunk=2)
    assert len(fb.classes) >= 2
    fb.run()
    torch.cuda.synchronize()
    for i in range(len(specs)):
        assert torch.equal(fb.output(i), ref[i]), i
    fb.reset()
    for i in range(len(specs)):
        fb.output(i).zero_()
    fb.capture_step()
    fb.replay_steps(5)
    torch.cuda.synchronize()
    _ = sum(float(fb.output(i).float().mean()) for i in range(len(specs)))   # eager work between replays
    fb.replay_steps(7)
    torch.cuda.synchronize()
    for i in range(len(specs)):
        st = fb.members[i]
        assert st._s.next_frame == 12 and st._s.emitted == 12
        assert torch.equal(fb.output(i), ref[i]), i
