"""Serving loop with continuous batching: independent streams arriving and leaving over time, the
frames of all admitted streams processed together in ticks (the real-time version of Section 6,
across streams).

Streams are grouped into classes (same frame size and parameters except the corner budget, seed and
stream id); each class is one ``StreamBatch`` on its own HIP stream (default priority), so the
classes of a tick overlap on the GPU. A tick takes the next buffered frame of every admitted stream
that has one, copies it from pinned host memory into the stream's device frame ring and runs one
``vs_batch_push`` per class: one launch per stage for all of the class's frames. Streams join and
leave between ticks, so requests that arrive while others are on the GPU are picked up by the next
tick.

Admission reserves a stream's device memory against an HBM budget from the exact sizes of its
buffers, before anything is allocated (plus the class's batch workspace when the class is new); a
stream that does not fit, or that would exceed the concurrency cap, waits in a FIFO queue with its
arriving frames buffered on the host, and is admitted, with all its frames, when a finished stream
releases memory. Each stream keeps its pyramids, points, fit state and trajectory on the device.
The buffers of a finished stream stay with its class (still counted against the budget) and are
reused by the next stream of that class, so admissions in steady state allocate nothing; pooled
buffers are released when a new stream needs their memory.
Streams share no state, so a stream's outputs are the same alone and in a mix (tested bit for bit).

``simulate`` replays a workload in virtual time: paced (frames submitted at their arrival times,
per-frame latency = completion of the tick that stabilized it minus its arrival; the host-to-device
copy is inside it) or saturated (all frames available at once, for capacity).
"""
from __future__ import annotations

import collections
import dataclasses
import gc
import math
import time

import numpy as np
import torch

from .params import SMOOTH_CAUSAL, SMOOTH_CENTERED, StabParams
from .pipeline import StreamBatch, member_bytes


@dataclasses.dataclass
class _Member:
    sid: int
    key: tuple
    P: StabParams
    width: int
    height: int
    reserved: int
    pending: collections.deque = dataclasses.field(default_factory=collections.deque)   # (j, host frame)
    received: int = 0
    closing: bool = False
    slot: int = -1
    stab: object = None


@dataclasses.dataclass
class _Class:
    batch: StreamBatch
    queue: torch.cuda.Stream
    reserved: int
    members: dict = dataclasses.field(default_factory=dict)    # slot -> _Member
    pool: list = dataclasses.field(default_factory=list)       # (Stabilizer, reserved bytes) of finished streams


def class_key(width: int, height: int, P: StabParams) -> tuple:
    """Streams whose keys are equal can share a batch: everything but the corner budget, the RANSAC
    seed and the stream id."""
    return (width, height, P.replace(max_corners=0, seed=0, stream_id=0))


class StreamServer:
    def __init__(self, hbm_budget: int, device="cuda", max_concurrent: int = 128, capacity: int = 3000,
                 detect_chunk: int = 8, ring_frames: int = 2):
        self.budget = int(hbm_budget)
        self.used = 0
        self.dev = torch.device(device)
        self.max_concurrent = max_concurrent
        self.capacity = capacity
        self.detect_chunk = detect_chunk
        self.ring_frames = ring_frames
        self.classes: dict = {}
        self.streams: dict = {}             # sid -> admitted _Member
        self.waiting: collections.deque = collections.deque()   # queued _Member
        self.ticks = 0
        self.items = 0

    # ---- admission ------------------------------------------------------------------------------
    def _lag(self, P: StabParams) -> int:
        return P.radius if P.smooth_mode == SMOOTH_CENTERED else 0

    def _member_bytes(self, m: _Member) -> int:
        lag = self._lag(m.P)
        return member_bytes(m.width, m.height, m.P, self.capacity, max(self.ring_frames, lag + 2), lag + 2)

    def _class_bytes(self, m: _Member) -> int:
        if m.key in self.classes:
            return 0
        sb_proto = StreamBatch.workspace_bytes(m.width, m.height, m.P, self.capacity, self.max_concurrent,
                                               self.detect_chunk)
        return sb_proto

    def _pooled(self, m: _Member) -> bool:
        cls = self.classes.get(m.key)
        return cls is not None and bool(cls.pool)

    def _fits(self, m: _Member) -> bool:
        if len(self.streams) >= self.max_concurrent:
            return False
        if self._pooled(m):
            return True                      # reuses a pooled stream's buffers (already counted)
        need = self._member_bytes(m) + self._class_bytes(m)
        if self.used + need <= self.budget:
            return True
        # release pooled buffers of other classes, and empty classes, until it fits
        for key, cls in list(self.classes.items()):
            while cls.pool and self.used + need > self.budget:
                _, b = cls.pool.pop()
                self.used -= b
            if not cls.members and not cls.pool and key != m.key:
                del self.classes[key]
                self.used -= cls.reserved
                need = self._member_bytes(m) + self._class_bytes(m)
        return self.used + need <= self.budget

    def prepare(self, width: int, height: int, P: StabParams, streams: int = 0) -> bool:
        """Creates the class of (width, height, P) ahead of its first stream, with ``streams`` pooled
        members, so that first admissions allocate nothing. Returns False if it does not fit."""
        m = _Member(-1, class_key(width, height, P), P, width, height, 0)
        need = self._class_bytes(m) + streams * self._member_bytes(m)
        if self.used + need > self.budget:
            return False
        self._ensure_class(m)
        cls = self.classes[m.key]
        lag = self._lag(P)
        with torch.cuda.stream(cls.queue):
            for _ in range(streams):
                b = self._member_bytes(m)
                cls.pool.append((cls.batch.member(P, ring=max(self.ring_frames, lag + 2)), b))
                self.used += b
        return True

    def _ensure_class(self, m: _Member):
        cb = self._class_bytes(m)
        if cb:
            q = torch.cuda.Stream(device=self.dev)
            with torch.cuda.stream(q):
                sb = StreamBatch(m.width, m.height, m.P.replace(max_corners=min(m.P.max_corners, self.capacity)),
                                 self.capacity, self.max_concurrent, self.detect_chunk, device=self.dev)
            self.classes[m.key] = _Class(sb, q, cb)
            self.used += cb

    def _admit(self, m: _Member):
        self._ensure_class(m)
        cls = self.classes[m.key]
        lag = self._lag(m.P)
        # the member's buffers live on the class's queue, which is the only stream using them
        with torch.cuda.stream(cls.queue):
            if cls.pool:
                m.stab, m.reserved = cls.pool.pop()
                m.stab.rebind(m.P)
            else:
                m.reserved = self._member_bytes(m)
                self.used += m.reserved
                m.stab = cls.batch.member(m.P, ring=max(self.ring_frames, lag + 2))
            m.slot = cls.batch.attach(m.stab)
        cls.members[m.slot] = m
        self.streams[m.sid] = m

    def open(self, sid, width: int, height: int, P: StabParams) -> bool:
        """Admit a stream if its state fits the budget and the concurrency cap (checked before
        allocating); otherwise queue it. Returns True if admitted now."""
        assert P.max_corners <= self.capacity and P.photometric_steps == 0
        m = _Member(sid, class_key(width, height, P), P, width, height, 0)
        if not self.waiting and self._fits(m):
            self._admit(m)
            return True
        self.waiting.append(m)
        return False

    def _find(self, sid) -> _Member:
        if sid in self.streams:
            return self.streams[sid]
        for m in self.waiting:
            if m.sid == sid:
                return m
        raise KeyError(sid)

    def submit(self, sid, frame_host: torch.Tensor):
        """Buffer one arriving frame (host uint8 [H, W], pinned, unchanged until processed)."""
        m = self._find(sid)
        assert not m.closing
        m.pending.append((m.received, frame_host))
        m.received += 1

    def close(self, sid):
        """No more frames: the stream ends once its buffered frames are processed."""
        self._find(sid).closing = True

    def has_work(self) -> bool:
        """Some admitted stream has a buffered frame or is closing (a tick would do something)."""
        return any(m.pending or m.closing for m in self.streams.values())

    # ---- ticks ----------------------------------------------------------------------------------
    def tick(self, timing: bool = False, on_emit=None) -> list:
        """One frame of every admitted stream that has one buffered, one batched push per class.
        Returns [(sid, frame index, event)] of the frames emitted; the event is recorded on the class's
        queue after the warps. ``on_emit(sid, frame index, output view)``, when given, is called for
        each with the class's queue current (work it enqueues there is ordered after the warp that
        wrote the view and before the view's memory is reused)."""
        out = []
        for cls in self.classes.values():
            items = [m for m in cls.members.values() if m.pending]
            if not items:
                continue
            ev = torch.cuda.Event(enable_timing=timing)
            with torch.cuda.stream(cls.queue):
                for m in items:
                    j, frame = m.pending.popleft()
                    ring = m.stab.ring
                    ring[j % ring.shape[0]].copy_(frame, non_blocking=True)
                res = cls.batch.push([m.slot for m in items], ready=ev)
                for m in items:
                    for e, view in res[m.slot]:
                        out.append((m.sid, e, ev))
                        if on_emit is not None:
                            on_emit(m.sid, e, view)
            self.ticks += 1
            self.items += len(items)
        out += self._finish(timing, on_emit)
        return out

    def _finish(self, timing: bool = False, on_emit=None) -> list:
        """Ends the closed streams whose frames are all processed (their buffers go to the class's
        pool) and admits queued streams that now fit."""
        out = []
        for m in [m for m in self.streams.values() if m.closing and not m.pending]:
            cls = self.classes[m.key]
            with torch.cuda.stream(cls.queue):
                st = cls.batch.detach(m.slot)
                em = st.flush()
                if em:
                    ev = torch.cuda.Event(enable_timing=timing)
                    ev.record()
                    for e, view in em:
                        out.append((m.sid, e, ev))
                        if on_emit is not None:
                            on_emit(m.sid, e, view)
            del cls.members[m.slot]
            del self.streams[m.sid]
            cls.pool.append((st, m.reserved))     # kept for the class's next stream, still reserved
            m.stab = None
        while self.waiting and self._fits(self.waiting[0]):
            self._admit(self.waiting.popleft())
        return out

    def drain(self, on_emit=None) -> list:
        """Ticks until every admitted stream is idle (closed ones finished, queued ones admitted)."""
        out = []
        while self.has_work():
            out += self.tick(on_emit=on_emit)
        if self.waiting and not self.streams:
            raise RuntimeError("a queued stream can never be admitted within the budget")
        return out

    def release_idle(self):
        """Frees pooled buffers and classes without streams (their memory leaves the budget)."""
        for key, cls in list(self.classes.items()):
            while cls.pool:
                _, b = cls.pool.pop()
                self.used -= b
            if not cls.members:
                del self.classes[key]
                self.used -= cls.reserved


@dataclasses.dataclass(frozen=True)
class ServedStream:
    sid: int
    arrival: float          # s (virtual time) of its first replayed frame
    n_frames: int
    fps: float
    width: int
    height: int
    params: StabParams
    clip: int               # index of the host frame pool this stream plays
    offset: int             # first frame of the pool


def poisson_workload(duration_s: float, rate: float, lifetime_s: tuple, fps: float, classes: list, k_range: tuple,
                     seed: int, max_concurrent: int = 128, warm_start_s: float = 0.0) -> list:
    """Seeded stream arrivals: Poisson(rate) over [-warm_start_s, duration), lifetimes U[lifetime_s],
    resolution drawn from ``classes`` [(width, height, levels, clip index)], corner budget U[k_range];
    the causal smoother (no lag). Streams beyond ``max_concurrent`` overlapping ones are dropped.
    With a warm start, streams that arrived before 0 enter the replay at 0 with their remaining frames,
    so the replay starts near the steady-state concurrency (rate x mean lifetime). Frames arriving at
    or after ``duration_s`` are cut, so a paced replay lasts ``duration_s``."""
    rng = np.random.default_rng(seed)
    t, out, sid = -warm_start_s, [], 0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration_s:
            break
        life = rng.uniform(*lifetime_s)
        w, h, levels, clip = classes[int(rng.integers(0, len(classes)))]
        k = int(rng.integers(k_range[0], k_range[1] + 1))
        offset = int(rng.integers(0, 1000))
        n = max(2, int(life * fps))
        active = sum(1 for s in out if s.arrival <= max(t, 0.0) < s.arrival + s.n_frames / s.fps)
        if active >= max_concurrent:
            continue
        P = StabParams(levels=levels, max_corners=k, smooth_mode=SMOOTH_CAUSAL, stream_id=sid, seed=1709 + sid)
        skip = int(math.ceil(-t * fps)) if t < 0 else 0   # frames played before the replay starts
        arr = t + skip / fps
        n = min(n - skip, int(math.ceil((duration_s - arr) * fps)))
        if n < 2:
            continue
        out.append(ServedStream(sid, arr, n, fps, w, h, P, clip, offset + skip))
        sid += 1
    return out


def simulate(server: StreamServer, workload: list, pools: list, paced: bool, max_inflight: int = 2,
             on_emit=None, measure_from: float = 0.0, keep_latencies: bool = False) -> dict:
    """Replay ``workload`` (ServedStream list) against ``server``. ``pools[clip]`` is a pinned host
    uint8 tensor [m, H, W] each stream plays cyclically from its offset. Ticks are issued whenever
    frames are buffered and fewer than ``max_inflight`` ticks are still running on the GPU, so the
    batch of a tick is whatever arrived while the previous ones ran. ``on_emit`` is passed to
    ``StreamServer.tick``. Returns per-frame latencies (paced; of the frames arriving at or after
    ``measure_from`` s, so a warm-up period can be left out) and throughput."""
    events = []             # (time, order, kind, stream, frame index): kind 0 = frame, 1 = end of stream
    for s in workload:
        for j in range(s.n_frames):
            events.append((s.arrival + j / s.fps, 0, s, j))
        events.append((s.arrival + (s.n_frames - 1) / s.fps, 1, s, s.n_frames))
    events.sort(key=lambda e: (e[0], e[2].sid, e[1], e[3]))
    for q in [c.queue for c in server.classes.values()]:
        q.synchronize()
    torch.cuda.synchronize()
    # the replay loop creates many short-lived objects: the cyclic garbage collector is paused during
    # it, as a serving loop would pause it, so its pauses do not land in the measured latencies
    gc_was_enabled = gc.isenabled()
    gc.disable()
    try:
        return _replay(server, events, pools, paced, max_inflight, on_emit, measure_from, keep_latencies)
    finally:
        if gc_was_enabled:
            gc.enable()


def _replay(server, events, pools, paced, max_inflight, on_emit, measure_from, keep_latencies) -> dict:
    arrival = {}
    done = []               # (arrival s, event)
    inflight = collections.deque()
    start = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record()
    i = 0
    n_out = 0
    max_conc = 0
    while True:
        now = (time.perf_counter() - t0) if paced else math.inf
        while i < len(events) and events[i][0] <= now:
            t, kind, s, j = events[i]
            i += 1
            if kind == 0:
                if j == 0:
                    server.open(s.sid, s.width, s.height, s.params)
                pool = pools[s.clip]
                server.submit(s.sid, pool[(s.offset + j) % pool.shape[0]])
                arrival[(s.sid, j)] = t
            else:
                server.close(s.sid)
        while inflight and all(e.query() for e in inflight[0]):
            inflight.popleft()
        if server.has_work() and len(inflight) < max_inflight:
            max_conc = max(max_conc, len(server.streams))
            emitted = server.tick(timing=True, on_emit=on_emit)
            evs = []
            for sid, e, ev in emitted:
                done.append((arrival[(sid, e)], ev))
                if not evs or evs[-1] is not ev:
                    evs.append(ev)
            n_out += len(emitted)
            if evs:
                inflight.append(evs)
            continue
        if i >= len(events) and not server.has_work():
            if server.waiting:
                raise RuntimeError("a queued stream can never be admitted within the budget")
            break
        if inflight and (not paced or i >= len(events) or server.has_work()):
            inflight[0][-1].synchronize()
        elif paced and i < len(events):
            lag = events[i][0] - (time.perf_counter() - t0)
            if lag > 0:
                time.sleep(min(lag, 0.002))
    torch.cuda.synchronize()            # every queue, also those of classes that have ended
    end = torch.cuda.Event(enable_timing=True)
    end.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_total_ms = start.elapsed_time(end)
    res = {"frames_out": n_out, "frames_in": len(arrival), "wall_s": wall, "gpu_s": gpu_total_ms / 1e3,
           "frames_per_s": n_out / max(gpu_total_ms / 1e3, 1e-9), "latency_ms_p50": None, "latency_ms_p99": None,
           "streams": len({e[2].sid for e in events}), "ticks": server.ticks, "mean_items_per_push": server.items / max(server.ticks, 1),
           "max_concurrent": max_conc}
    if paced and done:
        # completion on the GPU timeline (relative to the start event, recorded at t0) minus arrival
        arr = np.array([t for t, ev in done])
        lat = np.array([start.elapsed_time(ev) / 1e3 - t for t, ev in done])
        sel = lat[arr >= measure_from]
        res["latency_ms_p50"] = float(np.percentile(sel, 50) * 1e3)
        res["latency_ms_p99"] = float(np.percentile(sel, 99) * 1e3)
        res["latency_frames"] = int(sel.size)
        if keep_latencies:
            res["arrivals_s"] = arr
            res["latencies_s"] = lat
    return res
