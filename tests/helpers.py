"""Shared helpers of the GPU parity tests: device upload and pyramid-level extraction."""
import sys

import numpy as np
import torch


def dev(a) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def level_of(pyr: torch.Tensor, layout, l: int) -> np.ndarray:
    """Level l >= 1 of a device pyramid buffer as a host array."""
    off, p, w, h = layout.offset[l], layout.pitch[l], layout.width[l], layout.height[l]
    return pyr[off:off + p * h].view(h, p)[:, :w].cpu().numpy()


def say(*a):
    """Names the case on stdout before GPU work starts (flushed)."""
    print(*a, flush=True)
    sys.stdout.flush()


LK_DEFAULTS = dict(win_half=10, max_iter=30, eps=1e-3, min_eig=1e-2, fb=True, fb_thresh=1.0)


def lk_parity(g_xy, g_st, oracle_out, w, h, alive=None, tol=0.01, max_excluded=0.01, **prm):
    """Tracker parity of one frame pair (Section 3.2, Eqs. 3-6; Section 4.1 backward check).

    ``oracle_out`` is the oracle's (xy, status, fb_err, iters, eig_margin) for the same inputs.
    Statuses must agree except for points on a decision boundary: the oracle's round-trip error
    within 1e-3 relative of the backward-check threshold, its lambda_min / window size within 1e-3
    relative of the eigenvalue threshold at any level of either pass, a final position within 1 px
    of the image edge, or a pass that ran out of iterations at level 0. Positions of points valid on
    both sides must agree within ``tol``, except oracle tracks that ran out of iterations (their
    position is wherever the last update left a non-converging iteration). The exempted points are
    counted, reported and at most ``max_excluded`` of the tracked points (at least one allowed)."""
    prm = dict(LK_DEFAULTS, **prm)
    ro, rs, rf, it, mg = oracle_out
    n_alive = len(g_st) if alive is None else int(np.sum(alive))
    capped = (it[:, 0] >= prm["max_iter"]) | (it[:, 1] >= prm["max_iter"])
    classes = {
        "fb_band": np.abs(rf - prm["fb_thresh"]) <= 1e-3 * prm["fb_thresh"],
        "eig_band": mg <= 1e-3,
        "edge": (ro[:, 0] < 1) | (ro[:, 1] < 1) | (ro[:, 0] > w - 2) | (ro[:, 1] > h - 2),
        "iter_cap": capped,
    }
    boundary = np.zeros(len(g_st), bool)
    for v in classes.values():
        boundary |= v
    mism = (g_st != rs)
    unexplained = mism & ~boundary
    assert unexplained.sum() == 0, np.nonzero(unexplained)[0][:10]
    both = (g_st == 1) & (rs == 1)
    err = np.zeros(len(g_st))
    err[both] = np.abs(g_xy[both].astype(np.float64) - ro[both]).max(1)
    off = both & (err > tol)
    assert not (off & ~capped).any(), (err.max(), np.nonzero(off & ~capped)[0][:10])
    excluded = mism | off
    assert (both & ~excluded).sum() > 0
    r = dict(n=n_alive, compared=int((both & ~excluded).sum()), excluded=int(excluded.sum()),
             status_mismatch=int(mism.sum()), capped_beyond_tol=int(off.sum()),
             max_err=float(err[both & ~excluded].max()), **{"in_" + k: int(v.sum()) for k, v in classes.items()})
    assert r["excluded"] <= max(1, max_excluded * n_alive), r
    return r


def transform_err(p, q, w, h):
    """Largest distance between the images of the frame corners and centre under two centred
    similarities (a, b, tx, ty)."""
    cx, cy = (w - 1) / 2, (h - 1) / 2
    pts = np.array([[-cx, -cy], [cx, -cy], [-cx, cy], [cx, cy], [0, 0]])

    def ap(t):
        a, b, tx, ty = t
        return np.stack([a * pts[:, 0] - b * pts[:, 1] + tx, b * pts[:, 0] + a * pts[:, 1] + ty], 1)

    return float(np.max(np.hypot(*(ap(p) - ap(q)).T)))
