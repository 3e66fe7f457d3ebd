"""Benchmark of the stabilization hot path on one MI355X.

Workload: 1920x1080 uint8 synthetic UAV-like sequence of 600 frames (fBm terrain, jittery camera,
three independently moving squares), 1000 Shi-Tomasi corners, 5 pyramid levels, 21x21 LK window
with 30 iterations and the backward check, seeded RANSAC hybrid rigid/similarity fit, centred
moving-average smoothing (radius 15), bilinear warp. Frames are generated on the device and are
resident in HBM before timing.

One step = the whole hot path over the whole sequence through the segment-parallel sequence
path (pyramids, corners, tracking, fits, smoothing, warps of all 600 frames). Consecutive steps are
independent batches: by default they rotate over three stabilizer instances, one per HIP stream, so
one batch's launches fill the gaps of another's (each step does exactly the work of a serial step,
and every instance's outputs are checked equal to the serial run's). value = frames/s over the
timed steps (the median of three timed runs of --steps steps each); the serial ms per step (one
instance, one stream) is reported beside it. Also reported: the plain per-frame streaming path (throughput when frames
are pushed back to back, and per-frame compute latency p50/p99 when each frame is processed on
arrival), the roofline of the dominant kernel measured with HIP events on its stream, and the
CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# algorithmic FP32 work of the tracker per 21x21 window (point x level x direction): 8 kFLOP per
# window set-up and 5.3 kFLOP per Gauss-Newton iteration (about 18 and 12 FLOP per sample, an FMA
# counted as 2), the figures the roofline fraction is reported in.
LK_FLOP_SETUP = 8000.0
LK_FLOP_ITER = 5300.0
# the same work counted per operation of the method as written (a multiply and an add count 1 each):
# set-up: bilinear I (9), dI/dx and dI/dy (4 differences + 9 + 1 each), tensor products and sums
# (6); iteration: bilinear J (9), residual (1), two products and sums (4). Reported beside it.
LK_FLOP_SETUP_PER_SAMPLE = 43
LK_FLOP_ITER_PER_SAMPLE = 14
# the paper's own figure (context: another machine, another workload)
PAPER_FIGURE = {"fps": 50, "what": "Stage I (offline) average speed, motion estimation and trajectory smoothing "
                                  "(Table 2: 34.9 to 107.8 fps per video)",
                "hardware": "notebook with a dual-core 1.70 GHz CPU", "resolution": "320x240 to 640x480, 50 corners",
                "cite": "Abstract; Section 7.2, Table 2"}
FP32_VECTOR_PEAK_TFLOPS = 157.3
HBM_PEAK_GBS = 8000.0
# rocprofv3 summary of this workload (kernel trace + FETCH_SIZE / WRITE_SIZE passes)
PROFILE = os.path.join(ROOT, "profiles", "hd1080p_600f_sequence_path.md")
TRACKER_SOURCES = ("paper_1701_03572_amd/csrc/lk.hip", "paper_1701_03572_amd/csrc/vs_common.hpp")


def tracker_traffic_from_profile():
    """HBM bytes per tracker launch from the committed counter summary, or None when the summary is
    missing or was taken on other tracker sources (its recorded digest differs from the current one)."""
    import hashlib
    import re
    try:
        text = open(PROFILE).read()
    except OSError:
        return None
    m_bytes = re.search(r"Tracker HBM traffic per launch[^:]*: (\d+) bytes", text)
    m_dig = re.search(r"Tracker source digest[^:]*: ([0-9a-f]{16})", text)
    if not (m_bytes and m_dig):
        return None
    h = hashlib.sha256()
    for f in TRACKER_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return int(m_bytes.group(1)) if h.hexdigest()[:16] == m_dig.group(1) else None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def hbm_figures(V, ss, frames, P, n: int, W: int, H: int, ms_per_step: float) -> dict:
    """Achieved bandwidth of the HBM-bound launches (pyramid, warp) over all frames, timed with HIP
    events on the launch stream after the timed steps, and the whole step's algorithmic bytes over
    the step time. Algorithmic bytes per frame: pyramid = every level read once and every level above
    0 written once; warp = frame read + frame written; detection = one frame read every 5th frame;
    tracking = per level the window footprints of the K points (a (2h+3)^2 block on the set-up
    frame, (2h+2)^2 on the other), counted once and capped at the level size, doubled by the
    backward check."""
    import torch
    L = ss.layout
    sizes = [L.width[l] * L.height[l] for l in range(L.levels)]
    pyr_b = float(sum(sizes[:-1]) + sum(sizes[1:]))
    warp_b = 2.0 * W * H
    det_b = W * H / P.redetect_every
    w_set, w_oth = (2 * P.win_half + 3) ** 2, (2 * P.win_half + 2) ** 2
    lk_b = sum(min(s, P.max_corners * w_set) + min(s, P.max_corners * w_oth) for s in sizes) * (2 if P.fb else 1)
    fs = W * H

    def timed(fn, k=3):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(k):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / k

    pyr_ms = timed(lambda: V.vs_build_pyramid(frames, fs, ss.pyr, L.bytes, n, L))
    warp_ms = timed(lambda: V.vs_warp_frame(frames, fs, W, H, W, ss.mats, 6, ss.out, fs, W, n, P.border))
    per_frame = pyr_b + warp_b + det_b + lk_b

    def fig(b, ms):
        gbs = b * n / (ms / 1e3) / 1e9
        return {"bytes_per_frame": b, "ms": round(ms, 4), "achieved_gb_s": round(gbs, 1),
                "peak_gb_s": HBM_PEAK_GBS, "frac": round(gbs / HBM_PEAK_GBS, 4)}

    return {"pyramid": fig(pyr_b, pyr_ms), "warp": fig(warp_b, warp_ms),
            "step": dict(fig(per_frame, ms_per_step), parts_per_frame={"pyramid": pyr_b, "warp": warp_b,
                                                                        "detect": det_b, "track": lk_b})}


def differentiation_pass(V, ss, frames, P, n: int, W: int, H: int, steps: int) -> dict:
    """The differentiation pass of the 1080p workload over every pair of the sequence: the global
    photometric loss (vs_photometric_fwd) and its gradient, J^T J and J^T r in the 4 similarity
    parameters (vs_photometric_bwd) at each pair's fitted similarity, and the window loss of every one
    of the pair's 1000 features with its gradient in the 2 displacement components
    (vs_photometric_features, d = tracked - detected position). Timed with HIP events, median of 3
    runs of ``steps`` passes."""
    import numpy as np
    import torch
    from paper_1701_03572_amd import photometric as PH
    n_pairs = n - 1
    cap = ss.cap
    cx, cy, rho = PH.frame_geometry(W, H)
    m = P.photo_margin(W, H)
    omega = V.vs_rect(m, m, W - m, H - m)
    theta = PH.theta_from_fit(ss.pair_params[:n_pairs], W, H).contiguous()
    u = ss.src[:n_pairs].contiguous()
    d = (ss.dst[:n_pairs] - ss.src[:n_pairs]).contiguous()
    fs = W * H
    loss = torch.empty((n_pairs, V.VS_PHOTO_SUMS), dtype=torch.float64, device="cuda")
    sums = torch.empty_like(loss)
    wsb = V.vs_photometric_workspace(n_pairs, W, H)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    floss = torch.empty((n_pairs, cap), dtype=torch.float64, device="cuda")
    fgrad = torch.empty((n_pairs, cap, 2), dtype=torch.float64, device="cuda")

    def one():
        V.vs_photometric_fwd(frames, frames[1:], fs, W, H, W, n_pairs, theta, 4, cx, cy, rho, omega, loss, ws, wsb)
        V.vs_photometric_bwd(frames, frames[1:], fs, W, H, W, n_pairs, theta, 4, cx, cy, rho, omega, sums, ws, wsb)
        V.vs_photometric_features(frames, frames[1:], fs, W, H, W, n_pairs, u, d, cap, P.win_half, floss, fgrad)

    one()
    torch.cuda.synchronize()
    runs = []
    for _ in range(3):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(steps):
            one()
        b.record()
        torch.cuda.synchronize()
        runs.append(a.elapsed_time(b) / steps)
    ms = float(np.median(runs))
    px = (omega.x1 - omega.x0) * (omega.y1 - omega.y0)
    return {"what": "photometric loss and its backward over all %d pairs: global loss + dL/dtheta, J^T J, J^T r over "
                    "%dx%d pixels per pair, and %d features x 2 displacement gradients per pair (21x21 windows), "
                    "binary64" % (n_pairs, omega.x1 - omega.x0, omega.y1 - omega.y0, cap),
            "pairs": n_pairs, "features_per_pair": cap, "ms_per_pass": round(ms, 4),
            "runs_ms": [round(r, 4) for r in runs], "pairs_per_s": round(n_pairs / (ms / 1e3), 1),
            "pixels_per_s": round(2 * n_pairs * px / (ms / 1e3), 1)}


def run_batched(n_streams: int, n_frames: int, steps: int, warmup: int, cpu_frames: int = 0) -> dict:
    """Heterogeneous batch: n_streams independent streams of mixed resolution (320x240 .. 1920x1080),
    corner budget U[100, 2000] and 3-5 levels, all frames resident; one step stabilizes every frame of
    every stream. Timed eagerly and as a replayed HIP graph of the same step."""
    import torch
    from paper_1701_03572_amd import params, synth
    from paper_1701_03572_amd.batch import MultiStabilizer, StreamSpec

    specs, frames = [], []
    for s, (r, k, levels) in enumerate(synth.mixed_streams(n_streams, n_frames)):
        P = params.PRESETS["vga"].replace(levels=levels, max_corners=k, stream_id=s)
        specs.append(StreamSpec(r.width, r.height, n_frames, P))
        frames.append(synth.make_sequence(r, n_frames=n_frames, device="cuda").frames.contiguous())
    ms = MultiStabilizer(specs)
    for i, f in enumerate(frames):
        ms.load(i, f)
    total = ms.frames_total()

    def timed(fn, k):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record()
        for _ in range(k):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / k

    for _ in range(max(warmup, 1)):
        ms.run()
    eager_ms = timed(ms.run, steps)
    ms.capture_graph()
    ms.replay()
    graph_ms = timed(ms.replay, steps)
    res = {"workload": "%d streams x %d frames, resolution U{320x240, 640x480, 1280x720, 1920x1080}, corners "
                       "U[100, 2000], levels clamp(1 + floor(log2(W / 80)), 3, 5); Kalman smoothing" % (n_streams, n_frames),
           "streams": n_streams, "frames": total, "classes": len(ms.classes),
           "ms_per_step_eager": round(eager_ms, 4), "frames_per_s_eager": round(total / (eager_ms / 1e3), 1),
           "ms_per_step_graph": round(graph_ms, 4), "frames_per_s_graph": round(total / (graph_ms / 1e3), 1)}
    log("batched: %d streams, %d frames: eager %.2f ms/step (%.0f frames/s), graph %.2f ms/step (%.0f frames/s)" %
        (n_streams, total, eager_ms, res["frames_per_s_eager"], graph_ms, res["frames_per_s_graph"]))
    del ms
    torch.cuda.empty_cache()
    res["frame_step"] = run_frame_steps(specs, frames)
    del frames
    torch.cuda.empty_cache()
    if cpu_frames > 0:
        res["cpu_baseline"] = batched_cpu_baseline(n_streams, n_frames, cpu_frames)
        log("batched oracle: %.2f frames/s on %d threads" % (res["cpu_baseline"]["value"], res["cpu_baseline"]["cores"]))
    return res


def run_frame_steps(specs: list, frames: list) -> dict:
    """The same streams advanced frame by frame: each step is the next frame of all of them, one
    vs_batch_push per resolution class; timed eagerly and as replays of one captured step (one
    replay per frame step). Median of 3 passes over all frames."""
    import numpy as np
    import torch
    from paper_1701_03572_amd.batch import FrameStepBatch

    fb = FrameStepBatch(specs, frames, detect_chunk=16, keep_outputs=False)
    n = max(s.n_frames for s in specs)
    total = fb.frames_total()

    def timed(fn):
        runs = []
        for _ in range(3):
            fb.reset()
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            torch.cuda.synchronize()
            runs.append(a.elapsed_time(b))
        return float(np.median(runs))

    fb.reset()
    fb.run()                                   # warm-up pass
    eager_ms = timed(fb.run)
    fb.reset()
    fb.capture_step()
    fb.replay_steps(n)                         # warm-up pass of the graph
    graph_ms = timed(lambda: fb.replay_steps(n))
    res = {"what": "per-frame steps: each step the next frame of all %d streams, one batched launch set per class "
                   "(%d classes)" % (len(specs), len(fb.classes)),
           "steps": n, "ms_eager": round(eager_ms, 3), "frames_per_s_eager": round(total / (eager_ms / 1e3), 1),
           "ms_per_step_eager": round(eager_ms / n, 4), "ms_graph": round(graph_ms, 3),
           "frames_per_s_graph": round(total / (graph_ms / 1e3), 1), "ms_per_step_graph": round(graph_ms / n, 4)}
    log("frame-step batch: %d steps of %d streams: eager %.2f ms (%.0f frames/s), graph replays %.2f ms (%.0f frames/s)"
        % (n, len(specs), eager_ms, res["frames_per_s_eager"], graph_ms, res["frames_per_s_graph"]))
    del fb
    return res


def batched_cpu_baseline(n_streams: int, n_frames: int, cpu_frames: int) -> dict:
    """The oracle on a bounded sample of the same mix: the first ``cpu_frames`` frames of the first
    W streams, one stream per host thread (W = the host threads available, at most 16). The oracle is
    C behind ctypes, which releases the interpreter lock during each call, and keeps no global state,
    so the threads run in parallel."""
    import concurrent.futures as cf

    from oracle import oracle as O
    from paper_1701_03572_amd import params, synth

    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    mix = synth.mixed_streams(n_streams, n_frames)[:workers]
    jobs = []
    for s, (r, k, levels) in enumerate(mix):
        P = params.PRESETS["vga"].replace(levels=levels, max_corners=k, stream_id=s)
        jobs.append((synth.make_sequence(r, n_frames=cpu_frames).frames, P))
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(workers) as ex:
        list(ex.map(lambda j: O.stabilize(j[0], j[1]), jobs))
    wall = time.perf_counter() - t0
    return {"value": round(len(jobs) * cpu_frames / wall, 3), "unit": "frames/s", "cores": workers, "kind": "oracle",
            "sample": "first %d frames of the first %d streams of the same mix (%s), one stream per thread" %
                      (cpu_frames, len(jobs), ", ".join("%dx%d" % (r.width, r.height) for r, _, _ in mix))}


def run_serving(seconds: float) -> dict:
    """Serving with continuous batching: streams arrive as a Poisson process (2/s) and live U[10, 60] s
    at 30 fps, at most 128 at once; resolution U{640x480, 1280x720, 1920x1080, 3840x2160}, corner budget
    U[500, 3000], causal smoothing (no lag). A warm start (streams that arrived in the 60 s before the
    replay enter it with their remaining frames) puts the replay at the steady-state concurrency
    (about 2/s x 35 s = 70 streams) from its start. Frames come from pinned host memory (the
    host-to-device copy is inside the latency). Paced: frames submitted at their arrival times over
    ``seconds``, per-frame latency p50/p99. Saturated: the same frames all available at once, for
    capacity."""
    import torch
    from paper_1701_03572_amd import synth
    from paper_1701_03572_amd.serve import StreamServer, poisson_workload, simulate

    names = [("vga", 640, 480, 4), ("hd720", 1280, 720, 5), ("hd", 1920, 1080, 5), ("uhd", 3840, 2160, 5)]
    pools, classes = [], []
    for c, (name, w, h, levels) in enumerate(names):
        f = synth.make_sequence(synth.recipe(name, seed=1707 + c, motion="path"), n_frames=45, device="cuda").frames
        p = torch.empty(f.shape, dtype=torch.uint8, pin_memory=True)
        p.copy_(f)
        pools.append(p)
        classes.append((w, h, levels, c))
    wl = poisson_workload(seconds, 2.0, (10.0, 60.0), 30.0, classes, (500, 3000), seed=1708, max_concurrent=128,
                          warm_start_s=60.0)
    budget = 128 << 30

    from paper_1701_03572_amd.params import SMOOTH_CAUSAL, StabParams

    def server():
        # the classes and a pool of stream buffers are set up before the replay, as a deployed server's
        # would be, so admissions reuse buffers instead of allocating
        s = StreamServer(budget, capacity=3000, max_concurrent=128, detect_chunk=8)
        for w, h, levels, _ in classes:
            s.prepare(w, h, StabParams(levels=levels, max_corners=3000, smooth_mode=SMOOTH_CAUSAL), streams=40)
        torch.cuda.synchronize()
        return s

    # latency percentiles over the frames arriving after the first second: the warm start makes every
    # stream of the steady-state population begin at once (~70 first frames, each with a detection)
    paced = simulate(server(), wl, pools, paced=True, measure_from=1.0)
    sat = simulate(server(), wl, pools, paced=False)
    torch.cuda.empty_cache()
    res = {"workload": "Poisson arrivals 2/s, lifetimes U[10, 60] s at 30 fps, at most 128 concurrent (warm start: "
                       "the streams of the preceding 60 s join with their remaining frames), resolution U{640x480, "
                       "1280x720, 1920x1080, 3840x2160}, corners U[500, 3000], causal smoothing; frames from pinned "
                       "host memory; paced over %.0f s" % seconds,
           "streams": len(wl), "frames": paced["frames_out"], "concurrent_max": paced["max_concurrent"],
           "paced_latency_ms_p50": round(paced["latency_ms_p50"], 4),
           "paced_latency_ms_p99": round(paced["latency_ms_p99"], 4),
           "latency_over": "frames arriving after the first 1 s (%d frames)" % paced["latency_frames"],
           "paced_frames_per_s": round(paced["frames_out"] / paced["wall_s"], 1),
           "paced_mean_streams_per_push": round(paced["mean_items_per_push"], 2),
           "saturated_frames_per_s": round(sat["frames_per_s"], 1),
           "saturated_mean_streams_per_push": round(sat["mean_items_per_push"], 2),
           "hbm_budget_gib": budget >> 30, "batching": "continuous: one launch set per resolution class per tick"}
    log("serving: %d streams, %d frames, up to %d concurrent: paced latency p50 %.3f ms p99 %.3f ms (%.1f streams "
        "per push); saturated %.0f frames/s (%.1f streams per push)" %
        (len(wl), paced["frames_out"], paced["max_concurrent"], res["paced_latency_ms_p50"],
         res["paced_latency_ms_p99"], res["paced_mean_streams_per_push"], res["saturated_frames_per_s"],
         res["saturated_mean_streams_per_push"]))
    return res


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--frames", type=int, default=0, help="truncate the sequence (0: the full 600 frames)")
    ap.add_argument("--pipeline", type=int, default=3,
                    help="stabilizer instances, one per HIP stream, that consecutive steps rotate over so that "
                         "independent batches overlap (1: every step on one instance and the current stream)")
    ap.add_argument("--serial", action="store_true", help="same as --pipeline 1 (profiler runs)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--cpu-frames", type=int, default=6)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batched-streams", type=int, default=64)
    ap.add_argument("--batched-frames", type=int, default=120)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-diff", action="store_true", help="skip the differentiation pass timing")
    ap.add_argument("--no-hbm", action="store_true", help="skip the extra pyramid/warp launches of the HBM figures")
    ap.add_argument("--serving-seconds", type=float, default=20.0)
    ap.add_argument("--tuning", choices=["auto", "default", "cached"], default="auto",
                    help="launch tuning: autotune on the workload before timing (default), the library defaults, "
                         "or the cached choice for this class (--tuning-cache)")
    ap.add_argument("--tuning-cache", default=None, help="JSON cache of the autotuner (default: its per-user cache)")
    ap.add_argument("--tune-only", action="store_true", help="autotune, store the choice, print it and exit")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one elementwise kernel that reads and writes exactly 256 MiB (torch neg of "
                         "float32), the reference for scaling hardware byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: streams are independent and this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_1701_03572_amd import params, synth
    from paper_1701_03572_amd import vstab as V
    from paper_1701_03572_amd.pipeline import SequenceStabilizer, Stabilizer

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    V.load()
    rec = synth.RECIPES["hd"]
    P = params.PRESETS["hd"]
    n = rec.n_frames if args.frames <= 0 else min(args.frames, rec.n_frames)
    W, H = rec.width, rec.height
    log("generating %d frames of %dx%d on the device" % (n, W, H))
    t0 = time.time()
    seq = synth.make_sequence("hd", n_frames=n, device="cuda")
    frames = seq.frames.contiguous()
    torch.cuda.synchronize()
    log("generated in %.1f s" % (time.time() - t0))

    from paper_1701_03572_amd import tuning as T
    tuning = {"mode": args.tuning}
    ss = SequenceStabilizer(W, H, n, P)
    if args.tuning == "auto" or args.tune_only:
        # every candidate timed on the whole sequence step (ms per step in timings_ms)
        t, timings = T.autotune(frames, P.max_corners, P.levels, path=args.tuning_cache, reps=1, rounds=3,
                                step=lambda: ss.run(frames))
        tuning.update(choice=dataclasses.asdict(t), timings_ms={k: {c: round(v, 4) for c, v in d.items()}
                                                                 for k, d in timings.items()})
        log("autotuned launch choices: %s" % (t,))
        if args.tune_only:
            print(json.dumps(tuning))
            return 0
    elif args.tuning == "cached":
        t = T.apply(W, H, P.max_corners, args.tuning_cache)
        if t is None:
            print("no cached tuning for this class in %s" % (args.tuning_cache or T.default_cache_path()),
                  file=sys.stderr)
            return 2
        tuning["choice"] = dataclasses.asdict(t)
    else:
        T.set_tuning(None)
        tuning["choice"] = dataclasses.asdict(T.get_tuning())

    depth = 1 if args.serial else max(1, args.pipeline)
    inst = [ss] + [SequenceStabilizer(W, H, n, P) for _ in range(depth - 1)]
    queues = [torch.cuda.Stream() for _ in range(depth)]      # default priority

    def steps_serial(k, lk_events=None, work=None):
        for _ in range(k):
            ss.run(frames, lk_events=lk_events)
            if work is not None:
                work.append(ss.lk_work.clone())

    def steps_overlapped(k, first=0):
        # step j runs on instance (first + j) % depth, on that instance's stream: consecutive batches
        # share nothing but the read-only frames, so they overlap; each instance's own steps stay in order
        cur = torch.cuda.current_stream()
        for q in queues:
            q.wait_stream(cur)
        for j in range(k):
            m = (first + j) % depth
            with torch.cuda.stream(queues[m]):
                inst[m].run(frames)
        for q in queues:
            cur.wait_stream(q)

    def timed(fn, label):
        runs = []
        for r in range(3):
            torch.cuda.synchronize()
            t_start = torch.cuda.Event(enable_timing=True)
            t_end = torch.cuda.Event(enable_timing=True)
            t_start.record()
            fn()
            t_end.record()
            torch.cuda.synchronize()
            runs.append(t_start.elapsed_time(t_end))
            log("%s run %d: %.3f ms/step" % (label, r, runs[-1] / max(args.steps, 1)))
        return runs

    for i in range(args.warmup):
        if depth == 1:
            steps_serial(1)
        else:
            steps_overlapped(1, first=i)
        torch.cuda.synchronize()
        log("warmup step %d done" % i)
    if depth > 1 and args.warmup < depth:
        steps_overlapped(depth - args.warmup, first=args.warmup)    # every instance has run once
        torch.cuda.synchronize()
    # three timed runs of `steps` steps each; the reported figures are the median run's. With
    # depth > 1 the headline runs overlap consecutive batches over the instances and a serial set of
    # runs on one instance follows, which gives the tracker's per-launch durations (not stretched by
    # kernels of other streams) and the serial ms per step.
    wall0 = time.perf_counter()
    if depth > 1:
        runs_ms = timed(lambda: steps_overlapped(args.steps), "overlapped (%d streams)" % depth)
    wall = time.perf_counter() - wall0
    lk_events = []
    work = []
    serial_ms = timed(lambda: steps_serial(args.steps, lk_events, work), "serial")
    if depth == 1:
        runs_ms = serial_ms
        wall = time.perf_counter() - wall0
    if depth > 1:
        for m in range(1, depth):
            assert torch.equal(inst[m].out, ss.out) and torch.equal(inst[m].mats, ss.mats), \
                "instance %d of the overlapped runs differs from the serial run" % m
    ms_total = float(np.median(runs_ms))
    ms_per_step = ms_total / max(args.steps, 1)
    ms_per_step_serial = float(np.median(serial_ms)) / max(args.steps, 1)
    fps = n * args.steps / (ms_total / 1e3)
    log("sequence path: %.3f ms/step (median of 3 runs, %d stream(s)), %.0f frames/s; serial %.3f ms/step "
        "(wall of the headline runs %.3f s)" % (ms_per_step, depth, fps, ms_per_step_serial, wall))

    # roofline of the dominant kernel: the tracker (FP32 VALU bound)
    lk_ms = [a.elapsed_time(b) for a, b in lk_events]
    # [runs x steps, launches, segments, 2 or 3] -> [runs x steps, launches, 2 or 3]
    w = torch.stack(work).sum(dim=2).cpu().numpy()
    nwin = (2 * P.win_half + 1) ** 2
    setups, iters = float(w[..., 0].sum()), float(w[..., 1].sum())
    # set-ups formed: a backward track and the next pair's forward track share theirs
    formed = float(w[..., 2].sum()) if w.shape[-1] > 2 else setups
    n_launch = max(len(lk_ms), 1)
    flop_per_launch = (setups * LK_FLOP_SETUP + iters * LK_FLOP_ITER) / n_launch
    flop_per_launch_ops = (setups * LK_FLOP_SETUP_PER_SAMPLE + iters * LK_FLOP_ITER_PER_SAMPLE) * nwin / n_launch
    avg_lk_ms = float(np.mean(lk_ms)) if lk_ms else float("nan")
    achieved_tflops = flop_per_launch / (avg_lk_ms / 1e3) / 1e12
    achieved_ops = flop_per_launch_ops / (avg_lk_ms / 1e3) / 1e12
    lk_share = float(np.sum(lk_ms) / np.sum(serial_ms)) if serial_ms else float("nan")
    log("tracker: %.3f ms per launch avg, %.3e FLOP per launch, %.2f TFLOP/s (%.3f of peak), %.0f%% of the step" %
        (avg_lk_ms, flop_per_launch, achieved_tflops, achieved_tflops / FP32_VECTOR_PEAK_TFLOPS, 100 * lk_share))
    executed_tflops = (formed * LK_FLOP_SETUP + iters * LK_FLOP_ITER) / n_launch / (avg_lk_ms / 1e3) / 1e12
    kernel = "lk_segment_kernel7 (vs_track_lk_segments)"
    roofline = {"kernel": kernel, "bound": "alu",
                "achieved": round(achieved_tflops, 4),
                "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(achieved_tflops / FP32_VECTOR_PEAK_TFLOPS, 5),
                "traffic": tracker_traffic_from_profile(), "avg_launch_ms": round(avg_lk_ms, 4),
                "flop_per_launch": flop_per_launch,
                "flop_units": "8 kFLOP per window set-up, 5.3 kFLOP per iteration (point x level x direction)",
                "setups_per_launch": setups / n_launch, "iterations_per_launch": iters / n_launch,
                "launches_per_step": n_launch / max(len(work), 1),
                "setups_formed_per_launch": formed / n_launch,
                "achieved_formed": round(executed_tflops, 4),
                "frac_formed": round(executed_tflops / FP32_VECTOR_PEAK_TFLOPS, 5),
                "achieved_per_operation_count": round(achieved_ops, 4),
                "frac_per_operation_count": round(achieved_ops / FP32_VECTOR_PEAK_TFLOPS, 5),
                "share_of_step": round(lk_share, 4),
                "iterations_per_setup": iters / max(setups, 1.0)}

    hbm = None
    if not args.no_hbm:
        hbm = hbm_figures(V, ss, frames, P, n, W, H, ms_per_step)
        log("hbm: pyramid %.0f GB/s, warp %.0f GB/s; whole step %.2f MB/frame algorithmic, %.0f GB/s (%.3f of 8 TB/s)" %
            (hbm["pyramid"]["achieved_gb_s"], hbm["warp"]["achieved_gb_s"], hbm["step"]["bytes_per_frame"] / 1e6,
             hbm["step"]["achieved_gb_s"], hbm["step"]["frac"]))

    if args.calibrate_copy:
        a = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.neg(a, out=b)
        torch.cuda.synchronize()
        del a, b

    diff = None
    if not args.no_diff:
        diff = differentiation_pass(V, ss, frames, P, n, W, H, max(1, min(args.steps, 5)))
        log("differentiation pass: %.3f ms over %d pairs (%.0f pairs/s)" % (diff["ms_per_pass"], diff["pairs"],
                                                                            diff["pairs_per_s"]))

    plain = None
    if not args.no_plain:
        st = Stabilizer(W, H, P)
        for j in range(min(n, 40)):
            st.push(frames[j])
        st.flush()
        torch.cuda.synchronize()
        st.reset()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for j in range(n):
            st.push(frames[j])
        st.flush()
        e1.record()
        torch.cuda.synchronize()
        plain_ms = e0.elapsed_time(e1)
        plain_fps = n / (plain_ms / 1e3)
        # per-frame compute latency: each frame processed on arrival with an idle GPU, until the
        # outputs of its push are written (the push's ready event; the corner detection for the
        # next pair follows it)
        st.reset()
        lat = []
        for j in range(n):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            st.push(frames[j], ready=b)
            torch.cuda.synchronize()
            lat.append(a.elapsed_time(b))
        st.flush()
        torch.cuda.synchronize()
        lat = np.array(lat)
        plain = {"frames_per_s": round(plain_fps, 1), "ms_per_frame": round(plain_ms / n, 4),
                 "latency_ms_p50": round(float(np.percentile(lat, 50)), 4),
                 "latency_ms_p99": round(float(np.percentile(lat, 99)), 4),
                 "lag_frames": P.radius}
        log("plain path: %.0f frames/s, latency p50 %.3f ms p99 %.3f ms" % (plain_fps, plain["latency_ms_p50"],
                                                                           plain["latency_ms_p99"]))

    batched = None
    if not args.no_batched:
        batched = run_batched(args.batched_streams, args.batched_frames, args.steps, args.warmup,
                              0 if args.no_cpu_baseline else args.cpu_frames)

    serving = None
    if not args.no_serving:
        serving = run_serving(args.serving_seconds)

    cpu = None
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        k = max(2, min(args.cpu_frames, n))
        host = frames[:k].cpu().numpy()
        log("timing the CPU oracle on %d frames" % k)
        c0 = time.perf_counter()
        O.stabilize(host, P)
        c1 = time.perf_counter()
        cpu = {"value": round(k / (c1 - c0), 4), "unit": "frames/s", "cores": 1, "kind": "oracle",
               "sample": "first %d frames of the same 1920x1080 sequence, whole path (pyramids, corners, "
                         "tracking, fits, smoothing, warps), single-threaded binary64 C" % k}
        log("oracle: %.3f frames/s" % cpu["value"])

    out = {
        "metric": "stabilized frames/s at 1080p/1000 features vs plain path; p99 frame latency",
        "value": round(fps, 1),
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "runs_ms_per_step": [round(r / max(args.steps, 1), 4) for r in runs_ms],
        "ms_per_step_serial": round(ms_per_step_serial, 4),
        "overlapped_streams": depth,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "hd: 1920x1080 uint8, %d frames, 1000 corners, 5 levels, 21x21 LK x30 it + backward "
                               "check, RANSAC(128, 1 px) hybrid rigid/similarity, moving average r=15, bilinear warp" % n,
                   "path": "sequence (segment-parallel, one launch per stage per 5-frame step)" +
                           (", consecutive batches overlapped over %d instances on %d HIP streams" % (depth, depth)
                            if depth > 1 else ""),
                   "frames": n, "width": W, "height": H, "corners": P.max_corners, "levels": P.levels},
        "plain_path": plain,
        "differentiation_pass": diff,
        "batched": batched,
        "serving": serving,
        "tuning": tuning,
        "roofline": roofline,
        "hbm": hbm,
        "cpu_baseline": cpu,
        "paper": PAPER_FIGURE,
    }
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
