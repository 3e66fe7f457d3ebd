"""Stabilization pipelines over the C ABI (Section 2: motion estimation -> motion compensation ->
image composition).

``Stabilizer`` is the plain per-frame path of the real-time version (Section 6): every pushed
frame is processed as soon as it arrives and the output lags by the smoothing radius (centred
window) or not at all (causal / Kalman).

``SequenceStabilizer`` runs a whole resident sequence (the offline version, Stage I of the paper,
Section 7.1) with cross-frame parallelism: all pyramids in one launch, corner detection on every
5th frame in one launch, then one tracking launch that carries every point of every 5-frame segment
through the segment's pairs (re-detection and re-tracking after a skipped pair stay on the device
through gated launches), all fits, the smoothing and all warps in one launch each. Segments are independent because corners are
re-detected every 5 frames (Section 3.2), so both paths produce bit-identical results.

Every operation runs in libvstab's HIP kernels; torch only allocates device memory and supplies
the stream.
"""
from __future__ import annotations

import math

import torch

from . import vstab as V
from .params import StabParams


def _lk_params(P: StabParams) -> V.vs_lk_params:
    return V.vs_lk_params(P.win_half, P.max_iter, P.eps, P.min_eig, int(P.fb), P.fb_thresh)


def _detect_params(P: StabParams, w: int, h: int, max_corners: int | None = None,
                   k_items: torch.Tensor | None = None) -> V.vs_detect_params:
    mx, my = P.roi(w, h)
    k = P.max_corners if max_corners is None else max_corners
    return V.vs_detect_params(k, P.quality, P.min_dist, mx, my, None if k_items is None else k_items.data_ptr())


def _fit_params(P: StabParams, w: int, h: int) -> V.vs_fit_params:
    return V.vs_fit_params(P.model, P.ransac_iters, P.inlier_thresh, P.seed, P.stream_id, P.min_valid, P.dwell,
                           (w - 1) / 2.0, (h - 1) / 2.0)


def _smooth_params(P: StabParams, w: int, h: int) -> V.vs_smooth_params:
    return V.vs_smooth_params(P.smooth_mode, P.radius, P.kalman_ratio, P.crop, (w - 1) / 2.0, (h - 1) / 2.0)


class _PhotoRefiner:
    """Buffers and arguments of the optional photometric refinement of fitted pairs (in place, in
    the fit's (a, b, tx, ty) format; pairs the fit skipped stay unchanged)."""

    def __init__(self, P: StabParams, w: int, h: int, n_pairs_max: int, device):
        self.steps = P.photometric_steps
        self.W, self.H = w, h
        m = P.photo_margin(w, h)
        self.omega = V.vs_rect(m, m, w - m, h - m)
        self.cx, self.cy, self.rho = (w - 1) / 2.0, (h - 1) / 2.0, max(w, h) / 2.0
        n = max(n_pairs_max, 1)
        self.loss = torch.zeros((n, 2), dtype=torch.float64, device=device)
        self.accepted = torch.zeros(n, dtype=torch.int32, device=device)
        self.ws_bytes = V.vs_photometric_workspace(n, w, h)
        self.ws = _bytes(self.ws_bytes, device)

    def __call__(self, prev, nxt, frame_stride: int, n: int, pair_params, info, first_pair: int = 0):
        if self.steps <= 0 or n <= 0:
            return
        skip = info.data_ptr() + first_pair * V.FIT_INFO_BYTES + V.FIT_INFO_SKIPPED_OFFSET
        V.vs_photometric_refine(prev, nxt, frame_stride, self.W, self.H, self.W, n, pair_params, pair_params, 4,
                                V.VS_PHOTO_FIT, skip, V.FIT_INFO_BYTES // 4, self.cx, self.cy, self.rho, self.omega,
                                self.steps, self.loss, self.accepted, self.ws, self.ws_bytes)


def _bytes(n: int, device) -> torch.Tensor:
    return torch.empty(max(int(n), 1), dtype=torch.uint8, device=device)


def track_segments(o, f0: int, p0: int, fs: int, ps: int, pairs_of, P: StabParams, layout, lkp, dp, W: int, H: int,
                   work: torch.Tensor | None = None, lk_events: list | None = None, per_pair: bool = False) -> None:
    """Tracks every 5-frame segment of a resident sequence (or of a batch of sequences laid out on the
    same cadence): segment i starts at frame i * e (e = P.redetect_every) with the corners detected
    there, and its pairs (i e + s, i e + s + 1), s = 0 .. e - 1, are tracked in chain (Section 3.2),
    re-detecting on the device after a skipped pair. pairs_of(s) is the number of segments that have
    pair s (a prefix of the segments). ``o`` holds the point records (src, asrc, dst, status, fb_err:
    pair-major, capacity slots each), n_valid, the detection outputs (score, count) and the detection
    workspace (det_ws, det_ws_bytes).

    By default one vs_track_lk_segments call tracks every segment through all its pairs (one wave per
    point and segment), assuming that no pair is skipped; then, for s = 1 .. e - 1, the segments whose
    pair s - 1 was skipped detect frame s again and have their pairs from s on tracked again (both
    gated on the device by that pair's valid count). ``per_pair=True`` makes one vs_track_lk call per
    pair instead, each followed by the gated re-detection. Both give the same records. work: int64
    [1, segments, 3] (segment calls) or [e, segments, 2] (per-pair calls) counters of the first call;
    lk_events: (start, end) timing events around every tracking launch are appended."""
    e, cap = P.redetect_every, o.src.shape[1]
    xy, al, dst, st = o.src.data_ptr(), o.asrc.data_ptr(), o.dst.data_ptr(), o.status.data_ptr()
    fbe, nv = o.fb_err.data_ptr(), o.n_valid.data_ptr()
    rec2, rec1, rec4 = cap * 2 * 4, cap, cap * 4

    def timed_launch(fn):
        if lk_events is None:
            fn()
            return
        ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
        ev[0].record()
        fn()
        ev[1].record()
        lk_events.append(ev)

    def redetect(t: int, n_items: int):
        # re-detect frame t where pair t - 1 was skipped (too few valid points)
        V.vs_detect_corners(f0 + t * fs, e * fs, W, H, W, n_items, e, nv + (t - 1) * 4, P.min_valid, dp, cap,
                            xy + t * rec2, o.score.data_ptr() + t * cap * 8, o.count.data_ptr() + t * 4,
                            al + t * rec1, o.det_ws, o.det_ws_bytes)

    if not per_pair:
        n_seg = pairs_of(0)
        if n_seg <= 0:
            return
        last_pairs = sum(1 for s in range(e) if pairs_of(s) == n_seg)
        assert all(pairs_of(s) >= n_seg - 1 for s in range(e)), "only the last segment may be shorter"

        def segments(first: int, n_items: int, gate: int | None, wk):
            lp = last_pairs if n_items == n_seg else e
            V.vs_track_lk_segments(f0, p0, e * fs, e * ps, fs, ps, n_items, e, e, lp, first, layout, cap, lkp, xy,
                                   al, dst, st, fbe, nv, gate, P.min_valid, wk)

        timed_launch(lambda: segments(0, n_seg, None, work[0] if work is not None else None))
        for s in range(1, e):
            n_s = pairs_of(s)
            if n_s <= 0:
                break
            redetect(s, n_s)
            timed_launch(lambda: segments(s, n_s, nv + (s - 1) * 4, None))
        return
    for s in range(e):
        n_s = pairs_of(s)
        if n_s <= 0:
            break
        chained = s < e - 1
        timed_launch(lambda: V.vs_track_lk(
            f0 + s * fs, p0 + s * ps, f0 + (s + 1) * fs, p0 + (s + 1) * ps, e * fs, e * ps, n_s, e, layout,
            xy + s * rec2, al + s * rec1, cap, lkp, dst + s * rec2, st + s * rec1, fbe + s * rec4, nv + s * 4,
            xy + (s + 1) * rec2 if chained else None, al + (s + 1) * rec1 if chained else None,
            work[s] if work is not None else None))
        n_next = pairs_of(s + 1) if chained else 0
        if n_next > 0:
            redetect(s + 1, n_next)


class SequenceStabilizer:
    """Whole-sequence (offline) path with segment-parallel tracking. Buffers are allocated once
    for a (width, height, max_frames) shape and reused by every ``run``."""

    def __init__(self, width: int, height: int, max_frames: int, P: StabParams, device="cuda"):
        self.W, self.H, self.P = width, height, P
        self.n_max = max_frames
        self.dev = torch.device(device)
        self.layout = V.vs_pyramid_layout(width, height, width, P.levels)
        self.cap = P.max_corners
        n, cap, dev = max_frames, self.cap, self.dev
        self.n_seg_max = max(1, math.ceil((n - 1) / P.redetect_every))
        self.pyr = _bytes(n * self.layout.bytes, dev)
        self.src = torch.zeros((n, cap, 2), dtype=torch.float32, device=dev)      # one spare record
        self.asrc = torch.zeros((n, cap), dtype=torch.uint8, device=dev)
        self.dst = torch.zeros((n, cap, 2), dtype=torch.float32, device=dev)
        self.status = torch.zeros((n, cap), dtype=torch.uint8, device=dev)
        self.fb_err = torch.zeros((n, cap), dtype=torch.float32, device=dev)
        self.n_valid = torch.zeros(n, dtype=torch.int32, device=dev)
        self.count = torch.zeros(n, dtype=torch.int32, device=dev)
        self.score = torch.zeros((n, cap), dtype=torch.float64, device=dev)
        self.det_ws_bytes = V.vs_detect_workspace(width, height, self.n_seg_max)
        self.det_ws = _bytes(self.det_ws_bytes, dev)
        self.fit_ws_bytes = V.vs_fit_workspace(max(n - 1, 1), cap)
        self.fit_ws = _bytes(self.fit_ws_bytes, dev)
        self.fit_state = _bytes(V.FIT_STATE_BYTES, dev)
        self.pair_params = torch.zeros((max(n - 1, 1), 4), dtype=torch.float64, device=dev)
        self.info = _bytes(max(n - 1, 1) * V.FIT_INFO_BYTES, dev)
        self.inliers = torch.zeros((max(n - 1, 1), cap), dtype=torch.uint8, device=dev)
        # per-pair 2x3 models (a11, a12, tx, a21, a22, ty), centred; the smoother uses pair_params
        self.affine6 = torch.zeros((max(n - 1, 1), 6), dtype=torch.float64, device=dev)
        self.traj_state = _bytes(V.vs_traj_state_bytes(), dev)
        self.mats = torch.zeros((n, 6), dtype=torch.float64, device=dev)
        self.n_emitted = torch.zeros(1, dtype=torch.int32, device=dev)
        self.first = torch.zeros(1, dtype=torch.int64, device=dev)
        self.out = torch.empty((n, height, width), dtype=torch.uint8, device=dev)
        # per segment: [window set-ups, iterations, set-ups formed] of the tracking call
        self.lk_work = torch.zeros((1, self.n_seg_max, 3), dtype=torch.int64, device=dev)
        self._lkp = _lk_params(P)
        self._dp = _detect_params(P, width, height)
        self._fp = _fit_params(P, width, height)
        self._sp = _smooth_params(P, width, height)
        self.refine_pairs = _PhotoRefiner(P, width, height, n - 1, dev)

    def run(self, frames: torch.Tensor, warp: bool = True, lk_events: list | None = None) -> None:
        """Stabilize frames [n, H, W] (uint8, resident on the device). Results stay in the
        device buffers (pair_params, info, mats, out, ...); nothing is synchronised. When
        ``lk_events`` is a list, a (start, end) pair of timing events recorded on the current
        stream around every tracking launch is appended to it."""
        n = frames.shape[0]
        assert frames.is_cuda and frames.dtype == torch.uint8 and frames.is_contiguous()
        assert frames.shape[1:] == (self.H, self.W) and 1 <= n <= self.n_max
        P, L, cap = self.P, self.layout, self.cap
        fs, ps, e = self.H * self.W, L.bytes, P.redetect_every
        f0, p0 = frames.data_ptr(), self.pyr.data_ptr()
        V.vs_build_pyramid(f0, fs, p0, ps, n, L)
        n_pairs = n - 1
        if n_pairs >= 1:
            n_seg = math.ceil(n_pairs / e)
            xy, al = self.src.data_ptr(), self.asrc.data_ptr()
            V.vs_detect_corners(f0, e * fs, self.W, self.H, self.W, n_seg, e, None, 0, self._dp, cap, xy,
                                self.score.data_ptr(), self.count.data_ptr(), al, self.det_ws, self.det_ws_bytes)
            track_segments(self, f0, p0, fs, ps, lambda s: (n_pairs - 1 - s) // e + 1 if 0 <= s <= n_pairs - 1 else 0,
                           P, L, self._lkp, self._dp, self.W, self.H, self.lk_work, lk_events)
            V.vs_fit_state_init(self.fit_state)
            V.vs_fit_motion(self.src, self.dst, self.status, cap, n_pairs, self._fp, 0, self.fit_state,
                            self.pair_params, self.affine6, self.info, self.inliers, self.fit_ws, self.fit_ws_bytes)
            self.refine_pairs(f0, f0 + fs, fs, n_pairs, self.pair_params, self.info)
        V.vs_traj_state_init(self.traj_state)
        V.vs_smooth_trajectory(self.pair_params if n_pairs >= 1 else None, n_pairs, 1, self._sp, self.traj_state,
                               self.mats, n, self.n_emitted, self.first)
        if warp:
            V.vs_warp_frame(frames, fs, self.W, self.H, self.W, self.mats, 6, self.out, fs, self.W, n, P.border)

    def results(self, n: int) -> dict:
        """Host copies of the per-pair results of the last run over n frames."""
        n_pairs = n - 1
        return {
            "pair_params": self.pair_params[:n_pairs].cpu().numpy(),
            "info": V.fit_info_to_dicts(self.info[:n_pairs * V.FIT_INFO_BYTES]) if n_pairs > 0 else [],
            "mats": self.mats[:n].cpu().numpy(),
            "src": self.src[:n_pairs].cpu().numpy(),
            "alive_src": self.asrc[:n_pairs].cpu().numpy(),
            "dst": self.dst[:n_pairs].cpu().numpy(),
            "status": self.status[:n_pairs].cpu().numpy(),
            "fb_err": self.fb_err[:n_pairs].cpu().numpy(),
            "n_valid": self.n_valid[:n_pairs].cpu().numpy(),
            "inliers": self.inliers[:n_pairs].cpu().numpy(),
            "affine6": self.affine6[:n_pairs].cpu().numpy(),
        }


def stream_struct(width: int, height: int, P: StabParams, layout, capacity: int, out_slots: int) -> V.vs_stream:
    """A vs_stream with the geometry and parameters of a stream (no buffers)."""
    s = V.vs_stream()
    s.width, s.height, s.layout = width, height, layout
    s.detect, s.lk = _detect_params(P, width, height), _lk_params(P)
    s.fit, s.smooth = _fit_params(P, width, height), _smooth_params(P, width, height)
    s.capacity, s.redetect_every, s.min_valid, s.border = capacity, P.redetect_every, P.min_valid, P.border
    s.out_slots = out_slots
    s.photo_steps = max(P.photometric_steps, 0)
    return s


class Stabilizer:
    """Plain per-frame streaming path. ``push`` enqueues all work for one frame on the current
    stream through one native call (``vs_stream_push``) and returns the indices and output views of
    the frames it emits (the outputs are complete once the stream reaches this point). Pushed
    frames must stay unchanged until they are emitted; no frame is copied. The corner detection
    that serves the next pair is enqueued after the emitted frames' warps; a ``ready`` event given
    to ``push`` is recorded between the two, when the call's outputs are written."""

    def __init__(self, width: int, height: int, P: StabParams, device="cuda", out_slots: int | None = None,
                 capacity: int | None = None, ring=None):
        """capacity: point slots (default P.max_corners). ring: only for a stream advanced by a
        ``StreamBatch``: the number of frames of a device frame ring to allocate (frame j goes to
        ring[j % len]), or a uint8 device tensor [k, H, W] that already holds the stream's frames
        (frame j at [j % k], e.g. a resident sequence). Batch members need no workspaces of their own."""
        self.W, self.H, self.P = width, height, P
        self.dev = torch.device(device)
        dev = self.dev
        self.layout = V.vs_pyramid_layout(width, height, width, P.levels)
        self.cap = cap = capacity or P.max_corners
        self.batched = ring is not None
        self.pyr = _bytes(2 * self.layout.bytes, dev)
        self.pts = torch.zeros((2, cap, 2), dtype=torch.float32, device=dev)
        self.alive = torch.zeros((2, cap), dtype=torch.uint8, device=dev)
        self.dst = torch.zeros((cap, 2), dtype=torch.float32, device=dev)
        self.status = torch.zeros(cap, dtype=torch.uint8, device=dev)
        self.fb_err = torch.zeros(cap, dtype=torch.float32, device=dev)
        self.n_valid = torch.zeros(1, dtype=torch.int32, device=dev)
        self.count = torch.zeros(1, dtype=torch.int32, device=dev)
        self.det_ws_bytes = 0 if self.batched else V.vs_detect_workspace(width, height, 1)
        self.det_ws = None if self.batched else _bytes(self.det_ws_bytes, dev)
        self.fit_ws_bytes = 0 if self.batched else V.vs_fit_workspace(1, cap)
        self.fit_ws = None if self.batched else _bytes(self.fit_ws_bytes, dev)
        self.fit_state = _bytes(V.FIT_STATE_BYTES, dev)
        self.pair_params = torch.zeros((1, 4), dtype=torch.float64, device=dev)
        self.info = _bytes(V.FIT_INFO_BYTES, dev)
        self.inliers = torch.zeros(cap, dtype=torch.uint8, device=dev)
        self.affine6 = torch.zeros((1, 6), dtype=torch.float64, device=dev)   # last pair's 2x3 model
        self.traj_state = _bytes(V.vs_traj_state_bytes(), dev)
        self.lag = P.radius if P.smooth_mode == V.VS_SMOOTH_CENTERED else 0
        self.mats_cap = self.lag + 2
        self.mats = torch.zeros((self.mats_cap, 6), dtype=torch.float64, device=dev)
        self.n_emitted = torch.zeros(1, dtype=torch.int32, device=dev)
        self.first = torch.zeros(1, dtype=torch.int64, device=dev)
        self.out_slots = out_slots or (self.lag + 2)
        self.out = torch.empty((self.out_slots, height, width), dtype=torch.uint8, device=dev)
        self.refine_pair = None if self.batched else _PhotoRefiner(P, width, height, 1, dev)
        if isinstance(ring, int):
            ring = torch.empty((max(ring, self.lag + 2), height, width), dtype=torch.uint8, device=dev)
        self.ring = ring
        s = self._s = stream_struct(width, height, P, self.layout, cap, self.out_slots)
        for name in ("pyr", "pts", "alive", "dst", "status", "fb_err", "n_valid", "count", "fit_state", "pair_params",
                     "affine6", "info", "inliers", "traj_state", "mats", "n_emitted", "out"):
            setattr(s, name, getattr(self, name).data_ptr())
        s.first_frame = self.first.data_ptr()
        if self.batched:
            assert ring.is_cuda and ring.dtype == torch.uint8 and ring.is_contiguous() and ring.shape[1:] == (height, width)
            s.ring, s.ring_len = ring.data_ptr(), ring.shape[0]
        else:
            s.detect_ws, s.detect_ws_bytes = self.det_ws.data_ptr(), self.det_ws_bytes
            s.fit_ws, s.fit_ws_bytes = self.fit_ws.data_ptr(), self.fit_ws_bytes
            rp = self.refine_pair
            s.photo_omega = rp.omega
            s.photo_loss, s.photo_accepted = rp.loss.data_ptr(), rp.accepted.data_ptr()
            s.photo_ws, s.photo_ws_bytes = rp.ws.data_ptr(), rp.ws_bytes
        self.reset()

    def reset(self):
        V.vs_stream_reset(self._s)
        self.j = 0
        self.frames = {}           # frames pushed and not yet emitted (held alive for the device)

    def rebind(self, P: StabParams):
        """Reuse these buffers for a stream that differs only in its corner budget, RANSAC seed and
        stream id (same geometry, capacity and other parameters); call before it is (re)started."""
        assert P.replace(max_corners=0, seed=0, stream_id=0) == self.P.replace(max_corners=0, seed=0, stream_id=0)
        assert P.max_corners <= self.cap
        self.P = P
        self._s.detect.max_corners = P.max_corners
        self._s.fit.seed = P.seed
        self._s.fit.stream_id = P.stream_id

    def _collect(self, first: int, n: int) -> list:
        out = [(e, self.out[e % self.out_slots]) for e in range(first, first + n)]
        keep = min(first + n, self.j - 1)
        for e in [e for e in self.frames if e < keep]:
            del self.frames[e]
        return out

    def push(self, frame: torch.Tensor, ready: torch.cuda.Event | None = None) -> list:
        assert frame.is_cuda and frame.dtype == torch.uint8 and frame.shape == (self.H, self.W)
        assert frame.is_contiguous()
        self.frames[self.j] = frame
        handle = 0
        if ready is not None:
            if not ready.cuda_event:
                ready.record()          # creates the event; the push records it again
            handle = ready.cuda_event
        self._s.ready_event = handle
        first, n = V.vs_stream_push(self._s, frame)
        self.j += 1
        return self._collect(first, n)

    def flush(self) -> list:
        """End of stream: emit the frames still waiting for their smoothing window."""
        first, n = V.vs_stream_flush(self._s)
        out = [(e, self.out[e % self.out_slots]) for e in range(first, first + n)]
        self.frames.clear()
        return out


def _r512(n: int) -> int:
    return (max(int(n), 1) + 511) // 512 * 512


def member_bytes(width: int, height: int, P: StabParams, capacity: int, ring_frames: int, out_slots: int) -> int:
    """Device bytes of a batch member (a ``Stabilizer`` built with a ring of ``ring_frames`` frames),
    computed from the sizes of its buffers (each rounded to the allocator's 512-byte granule), so a
    server can reserve them before allocating anything."""
    layout = V.vs_pyramid_layout(width, height, width, P.levels)
    lag = P.radius if P.smooth_mode == V.VS_SMOOTH_CENTERED else 0
    cap = capacity
    plane = width * height
    sizes = [2 * layout.bytes, 16 * cap, 2 * cap, 8 * cap, cap, 4 * cap, 4, 4, V.FIT_STATE_BYTES, 32,
             V.FIT_INFO_BYTES, cap, 48, V.vs_traj_state_bytes(), (lag + 2) * 48, 4, 8, out_slots * plane,
             max(ring_frames, lag + 2) * plane]
    return sum(_r512(b) for b in sizes)


class StreamBatch:
    """Streams of one class (same frame size, capacity and parameters except the corner budget, seed
    and stream id) advanced together, one frame per stream per ``push``, with one launch per stage for
    all of them (vs_batch_push). Members are ``Stabilizer`` objects built with ``ring`` set and this
    batch's capacity; their outputs equal those of the same streams pushed alone, bit for bit."""

    def __init__(self, width: int, height: int, P: StabParams, capacity: int, max_streams: int,
                 detect_chunk: int = 8, device="cuda"):
        self.W, self.H, self.P, self.cap = width, height, P, capacity
        self.dev = torch.device(device)
        self.layout = V.vs_pyramid_layout(width, height, width, P.levels)
        lag = P.radius if P.smooth_mode == V.VS_SMOOTH_CENTERED else 0
        self.proto = stream_struct(width, height, P, self.layout, capacity, lag + 2)
        self.max_streams = max_streams
        self.detect_chunk = min(detect_chunk, max_streams)
        self.ws_bytes = V.vs_batch_workspace(self.proto, max_streams, self.detect_chunk)
        self.ws = _bytes(self.ws_bytes, self.dev)
        self.b = V.vs_batch()
        V.vs_batch_init(self.b, self.proto, max_streams, self.detect_chunk, self.ws, self.ws_bytes)
        self.members: dict = {}

    @staticmethod
    def workspace_bytes(width: int, height: int, P: StabParams, capacity: int, max_streams: int,
                        detect_chunk: int = 8) -> int:
        layout = V.vs_pyramid_layout(width, height, width, P.levels)
        lag = P.radius if P.smooth_mode == V.VS_SMOOTH_CENTERED else 0
        proto = stream_struct(width, height, P, layout, capacity, lag + 2)
        return _r512(V.vs_batch_workspace(proto, max_streams, min(detect_chunk, max_streams)))

    def free_slot(self) -> int | None:
        for i in range(self.max_streams):
            if i not in self.members:
                return i
        return None

    def member(self, P: StabParams, out_slots: int | None = None, ring=None) -> Stabilizer:
        """A new stream of this class (corner budget, seed and stream id from P), not yet attached."""
        if ring is None:
            ring = (P.radius if P.smooth_mode == V.VS_SMOOTH_CENTERED else 0) + 2
        return Stabilizer(self.W, self.H, P, device=self.dev, out_slots=out_slots, capacity=self.cap, ring=ring)

    def attach(self, st: Stabilizer, slot: int | None = None) -> int:
        slot = self.free_slot() if slot is None else slot
        assert slot is not None, "batch full"
        V.vs_batch_attach(self.b, slot, st._s)
        st.j = 0
        self.members[slot] = st
        return slot

    def detach(self, slot: int) -> Stabilizer:
        V.vs_batch_detach(self.b, slot)
        return self.members.pop(slot)

    def push(self, slots: list, ready: torch.cuda.Event | None = None) -> dict:
        """One frame of every listed stream (frame j of a stream must be in its ring at j % len).
        Returns {slot: [(frame index, output view), ...]} of the frames emitted."""
        handle = 0
        if ready is not None:
            if not ready.cuda_event:
                ready.record()
            handle = ready.cuda_event
        self.b.ready_event = handle
        first, cnt = V.vs_batch_push(self.b, list(slots))
        out = {}
        for sl, f, c in zip(slots, first, cnt):
            st = self.members[sl]
            st.j += 1
            out[sl] = [(e, st.out[e % st.out_slots]) for e in range(f, f + c)]
        return out

    def note_replayed(self, slots: list, steps: int):
        V.vs_batch_note_replayed(self.b, list(slots), steps)
        for sl in slots:
            self.members[sl].j += steps
