"""Run-to-run determinism of the six-stage path: the same frames give bit-identical results on a
second run of the same stabilizer and on a freshly built one (every cross-workgroup reduction on
this path has a fixed order; the photometric extension, whose sums use FP64 atomics, is not
enabled here).
"""
import numpy as np
import pytest
import torch

from helpers import dev, say
from paper_1701_03572_amd import params, synth
from paper_1701_03572_amd import vstab as V
from paper_1701_03572_amd.pipeline import SequenceStabilizer

pytestmark = pytest.mark.gpu


def run_once(ss, frames_dev, n):
    ss.run(frames_dev)
    torch.cuda.synchronize()
    r = ss.results(n)
    # the fit records as raw bytes: bit-exact, and their NaN fields (err_affine when the affine is
    # not a candidate) compare equal
    r["info"] = ss.info[:(n - 1) * V.FIT_INFO_BYTES].cpu().numpy()
    r["out"] = ss.out[:n].cpu().numpy()
    return r


def assert_same(a, b):
    for k in a:
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)


@pytest.mark.parametrize("name,n", [("tiny", 21), ("vga", 11)])
def test_sequence_runs_are_bit_identical(name, n):
    say("determinism", name, n)
    P = params.PRESETS[name]
    frames = synth.make_sequence(name, n_frames=n).frames
    h, w = frames.shape[1:]
    fd = dev(frames)
    ss = SequenceStabilizer(w, h, n, P)
    first = run_once(ss, fd, n)
    again = run_once(ss, fd, n)
    fresh = run_once(SequenceStabilizer(w, h, n, P), fd, n)
    assert_same(first, again)
    assert_same(first, fresh)
    assert sum(not i["skipped"] for i in V.fit_info_to_dicts(ss.info[:(n - 1) * V.FIT_INFO_BYTES])) > 0
