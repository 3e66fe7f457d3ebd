"""GPU parity of fit_similarity against the oracle (Section 4, Eq. 7; Section 4.1 hybrid switch
and skip rule): identical inlier sets, model choices and skip flags; parameters within 1e-4
relative (binary64 on both sides, two different least-squares routes)."""
import math

import numpy as np
import pytest
import torch

from helpers import dev, say
from oracle import oracle as O
from paper_1701_03572_amd import vstab as V

pytestmark = pytest.mark.gpu

W, H = 640, 480


def make_pairs(n_pairs, cap, seed, outlier_frac=0.3, noise=0.3, valid_frac=0.9, small=(), shear=0.0):
    rng = np.random.default_rng(seed)
    src = np.zeros((n_pairs, cap, 2), np.float32)
    dst = np.zeros((n_pairs, cap, 2), np.float32)
    valid = np.zeros((n_pairs, cap), np.uint8)
    for p in range(n_pairs):
        n = cap if p not in small else 6
        s = np.stack([rng.uniform(20, W - 20, n), rng.uniform(20, H - 20, n)], 1)
        th, sc = rng.normal(0, 0.02), 1 + rng.normal(0, 0.01)
        a, b = sc * math.cos(th), sc * math.sin(th)
        c = np.array([(W - 1) / 2, (H - 1) / 2])
        x = s - c
        d = np.stack([a * x[:, 0] - b * x[:, 1], b * x[:, 0] + a * x[:, 1]], 1) + c + rng.normal(0, 5, 2)
        d[:, 0] += shear * x[:, 1]
        d += rng.normal(0, noise, d.shape)
        bad = rng.random(n) < outlier_frac
        d[bad] += rng.uniform(-30, 30, (bad.sum(), 2))
        src[p, :n] = s
        dst[p, :n] = d
        valid[p, :n] = rng.random(n) < valid_frac
    return src, dst, valid


def gpu_fit(src, dst, valid, model, iters, pair0=0, state=None, seed=11, min_valid=10, dwell=20, with_affine=False):
    n, cap = valid.shape
    fp = V.vs_fit_params(model, iters, 1.0, seed, 3, min_valid, dwell, (W - 1) / 2, (H - 1) / 2)
    st = state if state is not None else torch.zeros(V.FIT_STATE_BYTES, dtype=torch.uint8, device="cuda")
    if state is None:
        V.vs_fit_state_init(st)
    out = torch.zeros((n, 4), dtype=torch.float64, device="cuda")
    info = torch.zeros(n * V.FIT_INFO_BYTES, dtype=torch.uint8, device="cuda")
    inl = torch.full((n, cap), 9, dtype=torch.uint8, device="cuda")
    wsb = V.vs_fit_workspace(n, cap)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    if with_affine:
        m6 = torch.full((n, 6), 7.0, dtype=torch.float64, device="cuda")
        V.vs_fit_motion(dev(src), dev(dst), dev(valid), cap, n, fp, pair0, st, out, m6, info, inl, ws, wsb)
        torch.cuda.synchronize()
        return out.cpu().numpy(), V.fit_info_to_dicts(info), inl.cpu().numpy(), st, m6.cpu().numpy()
    V.vs_fit_similarity(dev(src), dev(dst), dev(valid), cap, n, fp, pair0, st, out, info, inl, ws, wsb)
    torch.cuda.synchronize()
    return out.cpu().numpy(), V.fit_info_to_dicts(info), inl.cpu().numpy(), st


def oracle_fit(src, dst, valid, model, iters, pair0=0, state=None, seed=11, min_valid=10, dwell=20):
    fp = O.fit_params(model, iters, 1.0, seed, 3, min_valid, dwell, W, H)
    st = state if state is not None else O.new_hybrid_state()
    res = []
    for p in range(len(valid)):
        res.append(O.fit_pair_affine(src[p].astype(np.float64), dst[p].astype(np.float64), valid[p], fp, pair0 + p,
                                     st))
    return res, st


def near_tie(x, y):
    return abs(x - y) < 1e-12 * max(abs(x), abs(y))


def check(g, r, g6=None):
    """Bit-exact inlier sets, counts, skips and decisions (up to exact ties of the RMS errors, where
    either choice is correct); parameters within 1e-4 relative (binary64 on both sides, measured
    ~1e-10: the gate below is 1e-8)."""
    gp, gi, gm = g
    for p, (rp, r6, ri, rm) in enumerate(r):
        assert gi[p]["skipped"] == ri["skipped"] and gi[p]["n_valid"] == ri["n_valid"], p
        assert gi[p]["decided_here"] == ri["decided_here"], p
        tie = False
        if ri["decided_here"]:
            errs = [ri["err_rigid"], ri["err_sim"]] + ([ri["err_affine"]] if ri["err_affine"] == ri["err_affine"] else [])
            tie = any(near_tie(x, y) for i, x in enumerate(errs) for y in errs[i + 1:])
            gerrs = [gi[p]["err_rigid"], gi[p]["err_sim"]] + ([gi[p]["err_affine"]] if len(errs) == 3 else [])
            np.testing.assert_allclose(gerrs, errs, rtol=1e-9, atol=1e-9)    # px; exact fits leave ~1e-14
            if len(errs) == 2:
                assert gi[p]["err_affine"] != gi[p]["err_affine"], p          # NaN outside three-way decisions
        if tie:
            continue                     # an exact tie: either model is correct, the rest follows from it
        assert gi[p]["model"] == ri["model"], p
        assert gi[p]["n_inliers"] == ri["n_inliers"], p
        np.testing.assert_array_equal(gm[p], rm)
        np.testing.assert_allclose(gp[p], rp, rtol=1e-4, atol=1e-9)
        # much tighter in practice: both sides are binary64
        assert np.max(np.abs(gp[p] - rp)) < 1e-8 * max(1.0, np.max(np.abs(rp)))
        if g6 is not None:
            assert np.max(np.abs(g6[p] - r6)) < 1e-8 * max(1.0, np.max(np.abs(r6)))


@pytest.mark.parametrize("model", [V.VS_RIGID, V.VS_SIMILARITY, V.VS_HYBRID, V.VS_AFFINE, V.VS_HYBRID3])
@pytest.mark.parametrize("iters", [0, 128])
def test_models_and_ransac(model, iters):
    say("fit", model, iters)
    src, dst, valid = make_pairs(25, 300, 1 + model + iters, shear=0.02 if model >= V.VS_AFFINE else 0.0)
    g = gpu_fit(src, dst, valid, model, iters, with_affine=True)
    r, _ = oracle_fit(src, dst, valid, model, iters)
    check(g[:3], r, g[4])
    if model == V.VS_HYBRID3:
        assert g[1][0]["model"] == V.VS_AFFINE     # sheared motion: the affine is chosen
    # fit_similarity is fit_motion without the 2x3 output
    g2 = gpu_fit(src, dst, valid, model, iters)
    np.testing.assert_array_equal(g2[0], g[0])
    np.testing.assert_array_equal(g2[2], g[2])


def test_hybrid_blocks_skips_and_split_calls():
    say("fit hybrid blocks")
    small = {0, 20, 21, 33, 40}
    src, dst, valid = make_pairs(61, 500, 5, small=small)
    g = gpu_fit(src, dst, valid, V.VS_HYBRID, 64)
    r, _ = oracle_fit(src, dst, valid, V.VS_HYBRID, 64)
    check(g[:3], r)
    assert [i for i, d in enumerate(g[1]) if d["decided_here"]] == [1, 22, 41, 60]
    assert all(g[1][p]["skipped"] for p in small)
    # the same stream fed in uneven calls gives bit-identical results
    st = torch.zeros(V.FIT_STATE_BYTES, dtype=torch.uint8, device="cuda")
    V.vs_fit_state_init(st)
    parts = []
    for a, b in [(0, 1), (1, 19), (19, 25), (25, 61)]:
        parts.append(gpu_fit(src[a:b], dst[a:b], valid[a:b], V.VS_HYBRID, 64, pair0=a, state=st))
    np.testing.assert_array_equal(np.concatenate([p[0] for p in parts]), g[0])
    np.testing.assert_array_equal(np.concatenate([p[2] for p in parts]), g[2])
    split_info = sum([p[1] for p in parts], [])
    assert len(split_info) == len(g[1])
    for a, b in zip(split_info, g[1]):
        for k in a:
            assert a[k] == b[k] or (a[k] != a[k] and b[k] != b[k]), k     # equal, or both NaN


@pytest.mark.parametrize("dwell", [1, 3, 7])
@pytest.mark.parametrize("model", [V.VS_HYBRID, V.VS_HYBRID3])
def test_dwell_state_machine_random_skips_and_splits(dwell, model):
    """The block-parallel dwell resolution equals the oracle's pair-by-pair walk: random skip runs,
    several dwell lengths, the stream fed in calls of random lengths."""
    rng = np.random.default_rng(dwell * 10 + model)
    n_pairs = 47
    small = set(np.nonzero(rng.random(n_pairs) < 0.3)[0].tolist()) | {5, 6, 7}
    src, dst, valid = make_pairs(n_pairs, 64, 40 + dwell, small=small, shear=0.02 if model == V.VS_HYBRID3 else 0.0)
    r, _ = oracle_fit(src, dst, valid, model, 8, dwell=dwell)
    whole = gpu_fit(src, dst, valid, model, 8, dwell=dwell, with_affine=True)
    check(whole[:3], r, whole[4])
    st = torch.zeros(V.FIT_STATE_BYTES, dtype=torch.uint8, device="cuda")
    V.vs_fit_state_init(st)
    cuts = sorted(set([0, n_pairs] + rng.integers(1, n_pairs, 6).tolist()))
    infos = []
    for a, b in zip(cuts[:-1], cuts[1:]):
        part = gpu_fit(src[a:b], dst[a:b], valid[a:b], model, 8, pair0=a, state=st, dwell=dwell)
        infos += part[1]
        np.testing.assert_array_equal(part[0], whole[0][a:b])
    for p, (g, w) in enumerate(zip(infos, whole[1])):
        assert g["model"] == w["model"] and g["decided_here"] == w["decided_here"] and g["skipped"] == w["skipped"], p


def test_capacity_4096_and_exact_recovery():
    say("fit 4096")
    rng = np.random.default_rng(3)
    cap = 4096
    s = np.stack([rng.uniform(0, W, cap), rng.uniform(0, H, cap)], 1).astype(np.float32)
    c = np.array([(W - 1) / 2, (H - 1) / 2])
    a, b = 1.01 * math.cos(0.03), 1.01 * math.sin(0.03)
    x = s.astype(np.float64) - c
    d = (np.stack([a * x[:, 0] - b * x[:, 1], b * x[:, 0] + a * x[:, 1]], 1) + c + [4.0, -2.0]).astype(np.float32)
    v = np.ones((1, cap), np.uint8)
    g = gpu_fit(s[None], d[None], v, V.VS_SIMILARITY, 128)
    r, _ = oracle_fit(s[None], d[None], v, V.VS_SIMILARITY, 128)
    check(g[:3], r)
    np.testing.assert_allclose(g[0][0], [a, b, 4.0, -2.0], atol=1e-5)


def test_affine_edge_cases():
    say("fit affine edge cases")
    rng = np.random.default_rng(8)
    cap = 64
    src = np.zeros((4, cap, 2), np.float32)
    dst = np.zeros((4, cap, 2), np.float32)
    valid = np.zeros((4, cap), np.uint8)
    # pair 0: exactly three points; pair 1: collinear points (similarity fallback);
    # pair 2: two points (no affine hypothesis, least squares falls back); pair 3: coincident points
    src[0, :3] = [[100, 80], [420, 130], [260, 390]]
    t = np.linspace(0, 1, 40)
    src[1, :40] = np.stack([60 + 500 * t, 50 + 300 * t], 1)
    src[2, :2] = [[100, 100], [300, 200]]
    src[3, :12] = [200, 150]
    for p in range(4):
        dst[p] = src[p] * 1.01 + [2.0, -1.0] + rng.normal(0, 0.2, (cap, 2))
    valid[0, :3] = valid[1, :40] = valid[2, :2] = valid[3, :12] = 1
    for model in (V.VS_AFFINE, V.VS_HYBRID3):
        for iters in (0, 16):
            g = gpu_fit(src, dst, valid, model, iters, min_valid=2, with_affine=True)
            r, _ = oracle_fit(src, dst, valid, model, iters, min_valid=2)
            check(g[:3], r, g[4])
            if model == V.VS_AFFINE:
                np.testing.assert_array_equal(g[2][1, :40], 1)     # no 3-point hypothesis on a line
                m6 = g[4][1]
                assert m6[0] == m6[4] and m6[1] == -m6[3]           # the similarity fallback


def test_rejects_bad_arguments():
    src, dst, valid = make_pairs(1, 10, 0)
    with pytest.raises(V.VsError):
        gpu_fit(src, dst, valid, 7, 0)
    with pytest.raises(V.VsError):
        gpu_fit(src, dst, valid, V.VS_HYBRID3, 8192)
    with pytest.raises(V.VsError):
        gpu_fit(src, dst, valid, V.VS_HYBRID, 0, dwell=0)
