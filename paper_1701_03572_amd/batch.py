"""Many independent streams in one batch (heterogeneous batching), with optional HIP-graph replay.

Streams whose frame shape and launch-wide parameters agree form a class. The frames of a class's
streams share one buffer in which every stream starts at a slot that is a multiple of the
re-detection cadence e, so the 5-frame segments of all its streams are the items of the same
launches: pyramids, corner detection (each segment with its stream's corner budget), the tracking of
every segment through its pairs with device-side re-detection, and the warps run once per class. The slot after a stream's last
segment is padding: its segment gets a corner budget of 0 and its frames replicate the stream's last
frame, so it costs little and touches nothing of the stream. Fits and smoothing keep per-stream
state (dwell decisions, trajectory) and run once per stream. ``run`` enqueues everything on the
current stream without synchronising, so it can be captured once and replayed (``capture_graph``).

Every stream's results equal those of the same stream processed alone (SequenceStabilizer): the
per-item work is the same and nothing crosses streams.
"""
from __future__ import annotations

import dataclasses
import math

import torch

from . import vstab as V
from .params import StabParams
from .pipeline import _detect_params, _fit_params, _lk_params, _smooth_params, track_segments


@dataclasses.dataclass(frozen=True)
class StreamSpec:
    width: int
    height: int
    n_frames: int
    params: StabParams


def class_key(spec: StreamSpec) -> tuple:
    """Parameters one launch shares: frame shape and every non-per-stream path parameter."""
    P = spec.params
    return (spec.width, spec.height, P.levels, P.win_half, P.max_iter, P.eps, P.min_eig, P.fb, P.fb_thresh,
            P.quality, P.min_dist, P.roi(spec.width, spec.height), P.redetect_every, P.min_valid, P.border)


def _bytes(n: int, device) -> torch.Tensor:
    return torch.empty(max(int(n), 1), dtype=torch.uint8, device=device)


class _Class:
    def __init__(self, members: list, device):
        spec0 = members[0][1]
        W, H, P0 = spec0.width, spec0.height, spec0.params
        self.W, self.H, self.P0 = W, H, P0
        e = self.e = P0.redetect_every
        self.layout = V.vs_pyramid_layout(W, H, W, P0.levels)
        self.cap = cap = max(s.params.max_corners for _, s in members)
        self.streams = []                        # (stream index, spec, first slot, frames, segments)
        off = 0
        for si, spec in members:
            nseg = max(1, math.ceil((spec.n_frames - 1) / e))
            self.streams.append((si, spec, off, spec.n_frames, nseg))
            off += e * (nseg + 1)                # next stream starts on the cadence; the gap is padding
        self.slots = off
        self.n_items = off // e
        dev = device
        n = self.slots
        self.frames = torch.zeros((n, H, W), dtype=torch.uint8, device=dev)
        self.pyr = _bytes(n * self.layout.bytes, dev)
        self.src = torch.zeros((n, cap, 2), dtype=torch.float32, device=dev)
        self.asrc = torch.zeros((n, cap), dtype=torch.uint8, device=dev)
        self.dst = torch.zeros((n, cap, 2), dtype=torch.float32, device=dev)
        self.status = torch.zeros((n, cap), dtype=torch.uint8, device=dev)
        self.fb_err = torch.zeros((n, cap), dtype=torch.float32, device=dev)
        self.n_valid = torch.zeros(n, dtype=torch.int32, device=dev)
        self.count = torch.zeros(n, dtype=torch.int32, device=dev)
        self.score = torch.zeros((n, cap), dtype=torch.float64, device=dev)
        self.det_ws_bytes = V.vs_detect_workspace(W, H, self.n_items)
        self.det_ws = _bytes(self.det_ws_bytes, dev)
        # corner budget of every segment item (0 for the padding segments)
        k = torch.zeros(self.n_items, dtype=torch.int32)
        for si, spec, off, nf, nseg in self.streams:
            k[off // e: off // e + nseg] = spec.params.max_corners
        self.k_items = k.to(dev)
        self._dp = _detect_params(P0, W, H, cap, self.k_items)
        self._lkp = _lk_params(P0)
        # per-stream fit and smoothing state; outputs in slot-indexed arrays
        max_pairs = max(nf - 1 for _, _, _, nf, _ in self.streams)
        self.fit_ws_bytes = V.vs_fit_workspace(max(max_pairs, 1), cap)
        self.fit_ws = _bytes(self.fit_ws_bytes, dev)
        self.fit_state = [_bytes(V.FIT_STATE_BYTES, dev) for _ in self.streams]
        self.traj_state = [_bytes(V.vs_traj_state_bytes(), dev) for _ in self.streams]
        self.pair_params = torch.zeros((n, 4), dtype=torch.float64, device=dev)
        self.info = _bytes(n * V.FIT_INFO_BYTES, dev)
        self.inliers = torch.zeros((n, cap), dtype=torch.uint8, device=dev)
        self.mats = torch.zeros((n, 6), dtype=torch.float64, device=dev)
        self.mats[:, 0] = 1.0
        self.mats[:, 4] = 1.0                    # padding slots keep the identity
        self.n_emitted = torch.zeros(len(self.streams), dtype=torch.int32, device=dev)
        self.first = torch.zeros(len(self.streams), dtype=torch.int64, device=dev)
        self.out = torch.empty((n, H, W), dtype=torch.uint8, device=dev)
        self._fp = [_fit_params(spec.params, W, H) for _, spec, _, _, _ in self.streams]
        self._sp = [_smooth_params(spec.params, W, H) for _, spec, _, _, _ in self.streams]

    def load(self, i: int, frames: torch.Tensor):
        si, spec, off, nf, nseg = self.streams[i]
        self.frames[off:off + nf].copy_(frames)
        self.frames[off + nf:off + self.e * (nseg + 1)].copy_(frames[nf - 1:nf].expand(self.e * (nseg + 1) - nf, -1, -1))

    def run(self, warp: bool):
        e, cap, L = self.e, self.cap, self.layout
        fs, ps = self.H * self.W, L.bytes
        f0, p0 = self.frames.data_ptr(), self.pyr.data_ptr()
        V.vs_build_pyramid(f0, fs, p0, ps, self.slots, L)
        xy, al = self.src.data_ptr(), self.asrc.data_ptr()
        rec2, rec1 = cap * 2 * 4, cap
        ni = self.n_items
        V.vs_detect_corners(f0, e * fs, self.W, self.H, self.W, ni, e, None, 0, self._dp, cap, xy,
                            self.score.data_ptr(), self.count.data_ptr(), al, self.det_ws, self.det_ws_bytes)
        track_segments(self, f0, p0, fs, ps, lambda s: ni if 0 <= s < e else 0, self.P0, L, self._lkp, self._dp,
                       self.W, self.H)
        ib = V.FIT_INFO_BYTES
        for j, (si, spec, off, nf, nseg) in enumerate(self.streams):
            npairs = nf - 1
            if npairs >= 1:
                V.vs_fit_state_init(self.fit_state[j])
                V.vs_fit_similarity(xy + off * rec2, self.dst.data_ptr() + off * rec2,
                                    self.status.data_ptr() + off * rec1, cap, npairs, self._fp[j], 0, self.fit_state[j],
                                    self.pair_params.data_ptr() + off * 32, self.info.data_ptr() + off * ib,
                                    self.inliers.data_ptr() + off * rec1, self.fit_ws, self.fit_ws_bytes)
            V.vs_traj_state_init(self.traj_state[j])
            V.vs_smooth_trajectory(self.pair_params.data_ptr() + off * 32 if npairs >= 1 else None, npairs, 1,
                                   self._sp[j], self.traj_state[j], self.mats.data_ptr() + off * 48, nf,
                                   self.n_emitted.data_ptr() + j * 4, self.first.data_ptr() + j * 8)
        if warp:
            V.vs_warp_frame(f0, fs, self.W, self.H, self.W, self.mats, 6, self.out, fs, self.W, self.slots,
                            self.P0.border)


class MultiStabilizer:
    """Batched stabilization of independent streams (see the module docstring)."""

    def __init__(self, specs: list, device="cuda"):
        self.specs = list(specs)
        self.dev = torch.device(device)
        groups: dict = {}
        for i, spec in enumerate(self.specs):
            groups.setdefault(class_key(spec), []).append((i, spec))
        self.classes = [_Class(members, self.dev) for members in groups.values()]
        self.where = {}
        for c in self.classes:
            for j, (si, spec, off, nf, nseg) in enumerate(c.streams):
                self.where[si] = (c, j)
        self.graph = None

    def load(self, i: int, frames: torch.Tensor):
        """Stage stream i's frames [n, H, W] (uint8, on the device) into the batch buffers."""
        c, j = self.where[i]
        c.load(j, frames)

    def run(self, warp: bool = True):
        for c in self.classes:
            c.run(warp)

    def capture_graph(self, warp: bool = True):
        """Capture one batched step into a HIP graph (after an eager warm-up step on a side stream)."""
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            self.run(warp)
        torch.cuda.current_stream().wait_stream(side)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.run(warp)
        self.graph = g
        return g

    def replay(self):
        self.graph.replay()

    def frames_total(self) -> int:
        return sum(s.n_frames for s in self.specs)

    def output(self, i: int) -> torch.Tensor:
        c, j = self.where[i]
        si, spec, off, nf, nseg = c.streams[j]
        return c.out[off:off + nf]

    def results(self, i: int) -> dict:
        """Host copies of stream i's per-pair results."""
        c, j = self.where[i]
        si, spec, off, nf, nseg = c.streams[j]
        npairs = nf - 1
        info = V.fit_info_to_dicts(c.info[off * V.FIT_INFO_BYTES:(off + npairs) * V.FIT_INFO_BYTES]) if npairs else []
        return {"pair_params": c.pair_params[off:off + npairs].cpu().numpy(), "info": info,
                "mats": c.mats[off:off + nf].cpu().numpy(), "n_valid": c.n_valid[off:off + npairs].cpu().numpy()}


class FrameStepBatch:
    """The same kind of workload advanced frame by frame (the real-time version of Section 6 across
    streams): each step processes the next frame of every stream, one ``vs_batch_push`` per class
    (``pipeline.StreamBatch``): one launch per stage for the current frames of all of the class's
    streams. Every stream's frames stay resident (its frame ring is its whole sequence). Since a
    step's launches depend only on which streams it lists, one step over all streams (all of one
    length) can be captured and replayed once per frame (``capture_step`` / ``replay_steps``).
    Every stream's outputs equal those of the stream processed alone (and those of
    ``MultiStabilizer``), bit for bit."""

    def __init__(self, specs: list, frames: list, detect_chunk: int = 16, keep_outputs: bool = True,
                 device="cuda"):
        from .pipeline import StreamBatch
        from .serve import class_key as serve_key
        self.specs = list(specs)
        self.dev = torch.device(device)
        groups: dict = {}
        for i, spec in enumerate(self.specs):
            groups.setdefault(serve_key(spec.width, spec.height, spec.params), []).append(i)
        self.classes = []                       # (StreamBatch, [(stream index, slot)])
        self.members = {}
        for idx in groups.values():
            s0 = self.specs[idx[0]]
            cap = max(self.specs[i].params.max_corners for i in idx)
            sb = StreamBatch(s0.width, s0.height, s0.params.replace(max_corners=cap), cap, len(idx),
                             min(detect_chunk, len(idx)), device=self.dev)
            slots = []
            for i in idx:
                spec = self.specs[i]
                fr = frames[i]
                assert fr.shape == (spec.n_frames, spec.height, spec.width) and fr.is_contiguous()
                st = sb.member(spec.params, out_slots=spec.n_frames if keep_outputs else None, ring=fr)
                slots.append((i, sb.attach(st)))
                self.members[i] = st
            self.classes.append((sb, slots))
        self.queues = [torch.cuda.Stream(device=self.dev) for _ in self.classes]
        self.graph = None
        self._capture_advanced = False
        self.t = 0

    def _push_all(self, lists: list):
        """One push per class on the class's queue, forked from and joined to the current stream."""
        cur = torch.cuda.current_stream(self.dev)
        used = []
        for (sb, _), q, act in zip(self.classes, self.queues, lists):
            if not act:
                continue
            q.wait_stream(cur)
            with torch.cuda.stream(q):
                sb.push(act)
            used.append(q)
        for q in used:
            cur.wait_stream(q)

    def reset(self):
        """Every stream back to frame 0 (re-attached at its slot, which resets it)."""
        for sb, slots in self.classes:
            for i, sl in slots:
                st = sb.detach(sl)
                sb.attach(st, sl)
        self.t = 0
        self._capture_advanced = False

    def _active(self, slots) -> list:
        return [sl for i, sl in slots if self.t < self.specs[i].n_frames]

    def step(self):
        self._push_all([self._active(slots) for _, slots in self.classes])
        self.t += 1

    def run(self):
        """Every frame of every stream, step by step (eager)."""
        n = max(s.n_frames for s in self.specs)
        while self.t < n:
            self.step()

    def capture_step(self):
        """Capture one step over all streams (they must share one length) into a HIP graph. The
        capture advances the host progress by one step, the replays do the device work."""
        assert len({s.n_frames for s in self.specs}) == 1, "graph steps need streams of one length"
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self._push_all([[sl for _, sl in slots] for _, slots in self.classes])
        self.graph = g
        self._capture_advanced = True
        return g

    def replay_steps(self, k: int):
        """k replays of the captured step: the next k frames of every stream."""
        for _ in range(k):
            self.graph.replay()
        adv = k - 1 if self._capture_advanced else k     # the capture already advanced the host once
        self._capture_advanced = False
        for sb, slots in self.classes:
            sb.note_replayed([sl for _, sl in slots], adv)
        self.t += k

    def frames_total(self) -> int:
        return sum(s.n_frames for s in self.specs)

    def output(self, i: int) -> torch.Tensor:
        return self.members[i].out
