"""Serving loop: independent streams arriving over time, each stabilized frame by frame on the GPU.

Each admitted stream owns device-resident state (a streaming Stabilizer: pyramid ping-pong, point
records, fit and trajectory state, output slots) plus a small device ring for its incoming frames;
its frames arrive in host memory (pinned) and are copied to the ring on the stream's HIP stream, so
the measured latency includes the host-to-device copy. Streams are spread round-robin over a small
pool of HIP streams (default priority), so the mostly single-workgroup launches of different
streams run concurrently instead of queueing behind each other. Admission reserves each stream's device memory
against an HBM budget (measured when its state is built); a stream that does not fit waits in a FIFO
queue until memory is released. Streams never share state, so a stream's outputs do not depend on
what else is being served (tested: alone vs in a mix).

``simulate`` replays a workload in virtual time: paced (frames are submitted at their arrival times,
per-frame latency = completion of the frame's stabilized output on the GPU timeline minus its
arrival) or saturated (every frame submitted as fast as possible, for capacity).
"""
from __future__ import annotations

import collections
import dataclasses
import time

import numpy as np
import torch

from .params import SMOOTH_CAUSAL, StabParams
from .pipeline import Stabilizer


@dataclasses.dataclass
class _Stream:
    sid: int
    stab: Stabilizer
    ring: torch.Tensor
    reserved: int
    queue: torch.cuda.Stream
    pushed: int = 0


class StreamServer:
    def __init__(self, hbm_budget: int, device="cuda", queues: int = 4):
        self.budget = int(hbm_budget)
        self.used = 0
        self.dev = torch.device(device)
        self.streams: dict = {}
        self.waiting: collections.deque = collections.deque()
        self.rejected = 0
        self.queues = [torch.cuda.Stream(device=self.dev) for _ in range(max(1, queues))]
        self._next_queue = 0

    def _build(self, sid, width, height, P: StabParams) -> _Stream:
        q = self.queues[self._next_queue % len(self.queues)]
        self._next_queue += 1
        # the new state is initialised on the stream's own queue, after what the current stream
        # has enqueued so far
        q.wait_stream(torch.cuda.current_stream(self.dev))
        before = torch.cuda.memory_allocated(self.dev)
        with torch.cuda.stream(q):
            stab = Stabilizer(width, height, P, device=self.dev)
            ring = torch.empty((stab.lag + 2, height, width), dtype=torch.uint8, device=self.dev)
        reserved = torch.cuda.memory_allocated(self.dev) - before
        return _Stream(sid, stab, ring, reserved, q)

    def open(self, sid, width: int, height: int, P: StabParams) -> bool:
        """Admit a stream if its state fits the budget; otherwise queue it. Returns True if admitted."""
        st = self._build(sid, width, height, P)
        if self.used + st.reserved > self.budget:
            del st
            self.waiting.append((sid, width, height, P))
            return False
        self.used += st.reserved
        self.streams[sid] = st
        return True

    def submit(self, sid, frame_host: torch.Tensor, ready: torch.cuda.Event | None = None) -> list:
        """Copy one arriving frame (host, uint8 [H, W]) to the device and enqueue its processing.
        Returns (frame index, output view) for the frames this push emits; ``ready`` (optional) is
        recorded on the stream's queue once they are written."""
        st = self.streams[sid]
        with torch.cuda.stream(st.queue):
            slot = st.ring[st.pushed % st.ring.shape[0]]
            slot.copy_(frame_host, non_blocking=True)
            st.pushed += 1
            return st.stab.push(slot, ready=ready)

    def close(self, sid) -> list:
        """End a stream: emit what is left, release its memory and admit queued streams that now fit."""
        st = self.streams.pop(sid)
        with torch.cuda.stream(st.queue):
            out = st.stab.flush()
        self.used -= st.reserved
        admitted = []
        while self.waiting:
            wsid, w, h, P = self.waiting[0]
            probe = self._build(wsid, w, h, P)
            if self.used + probe.reserved > self.budget:
                break
            self.waiting.popleft()
            self.used += probe.reserved
            self.streams[wsid] = probe
            admitted.append(wsid)
        self.last_admitted = admitted
        return out


@dataclasses.dataclass(frozen=True)
class ServedStream:
    sid: int
    arrival: float          # s (virtual time)
    n_frames: int
    fps: float
    width: int
    height: int
    params: StabParams
    clip: int               # index of the host frame pool this stream plays
    offset: int             # first frame of the pool


def poisson_workload(duration_s: float, rate: float, lifetime_s: tuple, fps: float, classes: list, k_range: tuple,
                     seed: int, max_concurrent: int = 128) -> list:
    """Seeded stream arrivals: Poisson(rate) over [0, duration), lifetimes U[lifetime_s], resolution
    drawn from ``classes`` [(width, height, levels, clip index)], corner budget U[k_range]; the causal
    smoother (no lag). Streams beyond ``max_concurrent`` overlapping ones are dropped."""
    rng = np.random.default_rng(seed)
    t, out, sid = 0.0, [], 0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration_s:
            break
        life = rng.uniform(*lifetime_s)
        w, h, levels, clip = classes[int(rng.integers(0, len(classes)))]
        k = int(rng.integers(k_range[0], k_range[1] + 1))
        active = sum(1 for s in out if s.arrival <= t < s.arrival + s.n_frames / s.fps)
        if active >= max_concurrent:
            continue
        P = StabParams(levels=levels, max_corners=k, smooth_mode=SMOOTH_CAUSAL, stream_id=sid)
        out.append(ServedStream(sid, t, max(2, int(life * fps)), fps, w, h, P, clip, int(rng.integers(0, 1000))))
        sid += 1
    return out


def simulate(server: StreamServer, workload: list, pools: list, paced: bool) -> dict:
    """Replay ``workload`` (ServedStream list) against ``server``. ``pools[clip]`` is a pinned host
    uint8 tensor [m, H, W] each stream plays cyclically from its offset. Returns per-frame latencies
    (paced) and throughput."""
    events = []             # (time, kind, stream, frame index)
    for s in workload:
        for j in range(s.n_frames):
            events.append((s.arrival + j / s.fps, 0 if j < s.n_frames - 1 else 1, s, j))
    events.sort(key=lambda e: (e[0], e[2].sid, e[3]))
    done = []               # (arrival s, cuda event)
    start = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record()
    admitted_at = {}
    n_out = 0
    for t, kind, s, j in events:
        if paced:
            lag = t - (time.perf_counter() - t0)
            if lag > 0:
                time.sleep(lag)
        if j == 0:
            if not server.open(s.sid, s.width, s.height, s.params):
                continue
            admitted_at[s.sid] = t
        if s.sid not in server.streams:
            continue                                  # still queued: its frames are dropped until admitted
        pool = pools[s.clip]
        frame = pool[(s.offset + j) % pool.shape[0]]
        queue = server.streams[s.sid].queue
        ev = torch.cuda.Event(enable_timing=True)
        emitted = server.submit(s.sid, frame, ready=ev)   # recorded on the queue after the push's warps
        if kind == 1:
            emitted += server.close(s.sid)
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(queue)                          # after the flush's warps too
        if emitted:
            done.append((t, ev, len(emitted)))
            n_out += len(emitted)
    for q in server.queues:
        torch.cuda.current_stream().wait_stream(q)
    end = torch.cuda.Event(enable_timing=True)
    end.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_total_ms = start.elapsed_time(end)
    res = {"frames_out": n_out, "wall_s": wall, "gpu_s": gpu_total_ms / 1e3,
           "frames_per_s": n_out / max(gpu_total_ms / 1e3, 1e-9), "latency_ms_p50": None, "latency_ms_p99": None,
           "streams": len(workload), "admitted": len(admitted_at), "queued_or_rejected": len(workload) - len(admitted_at)}
    if paced and done:
        # completion on the GPU timeline (relative to the start event, recorded at t0) minus arrival
        lat = np.array([start.elapsed_time(ev) / 1e3 - t for t, ev, _ in done])
        res["latency_ms_p50"] = float(np.percentile(lat, 50) * 1e3)
        res["latency_ms_p99"] = float(np.percentile(lat, 99) * 1e3)
    return res
