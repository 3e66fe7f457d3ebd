"""The no-allocation fit entry point (vs_fit_motion_noalloc, static device scratch) against
vs_fit_motion with a caller workspace: the same kernels, so every output must be bit-identical.
Two calls in a row on the shared scratch, the second smaller than the first; a batch beyond the
scratch is rejected before any work is enqueued."""
import numpy as np
import pytest
import torch

from helpers import dev, say
from paper_1701_03572_amd import vstab as V
from test_gpu_fit import H, W, make_pairs

pytestmark = pytest.mark.gpu


def _outputs(n, cap):
    return (torch.full((n, 4), 5.0, dtype=torch.float64, device="cuda"),
            torch.full((n, 6), 7.0, dtype=torch.float64, device="cuda"),
            torch.full((n * V.FIT_INFO_BYTES,), 3, dtype=torch.uint8, device="cuda"),
            torch.full((n, cap), 9, dtype=torch.uint8, device="cuda"))


def _state():
    st = torch.zeros(V.FIT_STATE_BYTES, dtype=torch.uint8, device="cuda")
    V.vs_fit_state_init(st)
    return st


def _run(src, dst, valid, fp, pair0, noalloc):
    n, cap = valid.shape
    st = _state()
    out, m6, info, inl = _outputs(n, cap)
    if noalloc:
        before = torch.cuda.memory_allocated()
        V.vs_fit_motion_noalloc(src, dst, valid, cap, n, fp, pair0, st, out, m6, info, inl)
        assert torch.cuda.memory_allocated() == before
    else:
        wsb = V.vs_fit_workspace(n, cap)
        ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
        V.vs_fit_motion(src, dst, valid, cap, n, fp, pair0, st, out, m6, info, inl, ws, wsb)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in (out, m6, info, inl, st)]


@pytest.mark.parametrize("model", [V.VS_HYBRID3, V.VS_HYBRID])
def test_noalloc_equals_workspace_call_twice(model):
    cases = [(48, 1000, 5), (7, 300, 6)]           # the second call is smaller (pairs and capacity)
    for n, cap, seed in cases:
        say("noalloc fit: model %d, %d pairs, capacity %d" % (model, n, cap))
        src, dst, valid = make_pairs(n, cap, seed, small=(2,))
        fp = V.vs_fit_params(model, 128, 1.0, 17, 2, 10, 20, (W - 1) / 2, (H - 1) / 2)
        s, d, v = dev(src), dev(dst), dev(valid)
        got = _run(s, d, v, fp, 3, noalloc=True)
        ref = _run(s, d, v, fp, 3, noalloc=False)
        for k, (g, r) in enumerate(zip(got, ref)):
            assert np.array_equal(g.view(np.uint8), r.view(np.uint8)), "output %d differs" % k
        info = V.fit_info_to_dicts(torch.from_numpy(got[2]))
        assert sum(i["skipped"] for i in info) == 1 and all(i["n_inliers"] > 0 for i in info if not i["skipped"])


def test_noalloc_rejects_oversize_batch():
    cap = 1000
    m = V.vs_fit_noalloc_max_pairs(cap)
    assert m == min(65535, V.VS_FIT_NOALLOC_SCRATCH_BYTES // V.vs_fit_workspace(1, cap)) and m >= 600
    assert V.vs_fit_noalloc_max_pairs(0) == 0 and V.vs_fit_noalloc_max_pairs(V.VS_MAX_CORNERS + 1) == 0
    n = m + 1
    say("noalloc fit: oversize batch of %d pairs" % n)
    valid = torch.zeros((n, cap), dtype=torch.uint8, device="cuda")
    pts = torch.zeros((n, cap, 2), dtype=torch.float32, device="cuda")
    fp = V.vs_fit_params(V.VS_SIMILARITY, 16, 1.0, 1, 0, 10, 20, 0.0, 0.0)
    st = _state()
    out, m6, info, inl = _outputs(n, cap)
    with pytest.raises(V.VsError, match="scratch"):
        V.vs_fit_motion_noalloc(pts, pts, valid, cap, n, fp, 0, st, out, m6, info, inl)
    torch.cuda.synchronize()
    assert bool((out == 5.0).all()) and bool((inl == 9).all())    # nothing was enqueued

