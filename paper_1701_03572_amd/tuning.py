"""Launch-shape autotuner.

The library's speed-only launch choices (``vs_set_tuning``: per-XCD mapping thresholds of the
pyramid, tracking and warp launches, points per tracking workgroup, the corner response's wave
segment height and the fit's hypothesis workgroups in flight) never change a result bit. ``autotune`` times the candidates of each kernel family on a batch of the caller's class and
keeps the fastest; the choice is cached in a JSON file keyed by GPU architecture, resolution class
and corner-budget class, and ``apply`` installs a cached choice before a run.
"""
from __future__ import annotations

import dataclasses
import json
import os

import torch

from . import vstab as V

RES_CLASSES = [(320, 240), (640, 480), (1280, 720), (1920, 1080), (3840, 2160)]
K_CLASSES = [256, 1024, 4096]
XCD_CANDIDATES = [1, 8, 65536]        # always, from 8 items (the default), never
LK_PPG_CANDIDATES = [1, 2, 4]
DET_ROWS_CANDIDATES = [0, 12, 30, 60, 120]   # 0: by batch size (the default)
FIT_GROUPS_CANDIDATES = [512, 1024, 2048, 4096, 8192]
MARGIN = 0.015                        # a candidate replaces the default only if this much faster


@dataclasses.dataclass(frozen=True)
class Tuning:
    xcd_pyramid: int = 8
    xcd_lk: int = 8
    xcd_warp: int = 8
    lk_ppg: int = 1
    det_rows: int = 0
    fit_groups: int = 2048

    def to_c(self) -> V.vs_tuning:
        return V.vs_tuning(self.xcd_pyramid, self.xcd_lk, self.xcd_warp, self.lk_ppg, self.det_rows, self.fit_groups)

    @staticmethod
    def from_c(t: V.vs_tuning) -> "Tuning":
        return Tuning(t.xcd_min_items_pyramid, t.xcd_min_items_lk, t.xcd_min_items_warp, t.lk_points_per_group,
                      t.detect_segment_rows, t.fit_groups_in_flight)


def set_tuning(t: Tuning | None):
    """Install ``t`` process-wide (None: the defaults)."""
    V.vs_set_tuning(None if t is None else t.to_c())


def get_tuning() -> Tuning:
    return Tuning.from_c(V.vs_get_tuning())


def resolution_class(w: int, h: int) -> str:
    for cw, ch in RES_CLASSES:
        if w * h <= cw * ch:
            return "%dx%d" % (cw, ch)
    return ">%dx%d" % RES_CLASSES[-1]


def k_class(k: int) -> str:
    for c in K_CLASSES:
        if k <= c:
            return "K<=%d" % c
    return "K>%d" % K_CLASSES[-1]


def cache_key(arch: str, w: int, h: int, k: int) -> str:
    return "%s/%s/%s" % (arch, resolution_class(w, h), k_class(k))


def device_arch(device=0) -> str:
    return torch.cuda.get_device_properties(device).gcnArchName.split(":")[0]


def default_cache_path() -> str:
    return os.environ.get("VS_TUNING_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "paper_1701_03572_amd", "tuning.json"))


def load_cache(path: str | None = None) -> dict:
    path = path or default_cache_path()
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def store(key: str, t: Tuning, timings: dict, workload: dict, path: str | None = None):
    path = path or default_cache_path()
    cache = load_cache(path)
    cache[key] = {"tuning": dataclasses.asdict(t), "timings_ms": timings, "workload": workload}
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def lookup(arch: str, w: int, h: int, k: int, path: str | None = None) -> Tuning | None:
    e = load_cache(path).get(cache_key(arch, w, h, k))
    return Tuning(**e["tuning"]) if e else None


def apply(w: int, h: int, k: int, path: str | None = None) -> Tuning | None:
    """Install the cached choice for this class on the current device, if there is one."""
    t = lookup(device_arch(), w, h, k, path)
    if t is not None:
        set_tuning(t)
    return t


def _time(fn, reps: int) -> float:
    fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def _compare(cands: dict, fn, reps: int, rounds: int) -> dict:
    """Median time (ms per call) of fn under each candidate tuning. The candidates are interleaved
    over ``rounds`` rounds in a rotating order, so clock ramps and drift are shared fairly."""
    names = list(cands)
    samples = {k: [] for k in names}
    for r in range(rounds):
        for i in range(len(names)):
            k = names[(i + r) % len(names)]
            set_tuning(cands[k])
            samples[k].append(_time(fn, reps))
    return {k: sorted(v)[len(v) // 2] for k, v in samples.items()}


def _pick(times: dict, default: str) -> str:
    """The fastest candidate, unless it beats the default by less than MARGIN."""
    best = min(times, key=times.get)
    return best if times[best] < times[default] * (1.0 - MARGIN) else default


def autotune(frames: torch.Tensor, k: int, levels: int, win_half: int = 10, reps: int = 3, rounds: int = 5,
             path: str | None = None, save: bool = True, step=None) -> tuple[Tuning, dict]:
    """Times every candidate of each kernel family on ``frames`` (uint8 [n, H, W] on the device,
    n >= 2, consecutive frames of one stream) and returns the fastest choice with the timings; a
    candidate must beat the default by MARGIN to replace it. With ``step`` (a callable that enqueues
    one whole pipeline step on these frames) every candidate is timed on that step, which counts
    the effects between kernels (cache state left by one launch for the next); otherwise each family
    is timed on its own kernel, the tracker on the pairs (frame j, frame j + 1) of every 5th frame
    from the corners of frame j. Leaves the chosen tuning installed; stores it in the cache with
    ``save``."""
    n, h, w = frames.shape
    frames = frames.contiguous()
    layout = V.vs_pyramid_layout(w, h, w, levels)
    fs, ps = h * w, max(layout.bytes, 1)
    pyr = torch.empty((n, ps), dtype=torch.uint8, device=frames.device)
    seg = max(1, (n - 1) // 5)
    base = Tuning()
    timings = {}

    # pyramid
    pyr_fn = lambda: V.vs_build_pyramid(frames, fs, pyr, ps, n, layout)
    timings["pyramid"] = _compare({str(x): dataclasses.replace(base, xcd_pyramid=x) for x in XCD_CANDIDATES},
                                  step or pyr_fn, reps, rounds)
    best_pyr = int(_pick(timings["pyramid"], str(base.xcd_pyramid)))
    set_tuning(dataclasses.replace(base, xcd_pyramid=best_pyr))
    pyr_fn()

    # tracker: corners of every segment start, then one tracking launch over the segments
    dp = V.vs_detect_params(k, 0.01, 10, max(16, w // 20), max(16, h // 20))
    xy = torch.zeros((n, k, 2), dtype=torch.float32, device=frames.device)
    al = torch.zeros((n, k), dtype=torch.uint8, device=frames.device)
    cnt = torch.zeros(n, dtype=torch.int32, device=frames.device)
    wsb = V.vs_detect_workspace(w, h, seg)
    ws = torch.empty(wsb, dtype=torch.uint8, device=frames.device)
    V.vs_detect_corners(frames, 5 * fs, w, h, w, seg, 5, None, 0, dp, k, xy, None, cnt, al, ws, wsb)
    lkp = V.vs_lk_params(win_half, 30, 1e-3, 1e-2, 1, 1.0)
    dst = torch.zeros((n, k, 2), dtype=torch.float32, device=frames.device)
    st = torch.zeros((n, k), dtype=torch.uint8, device=frames.device)
    f0, p0 = frames.data_ptr(), pyr.data_ptr()
    lk_fn = lambda: V.vs_track_lk(f0, p0, f0 + fs, p0 + ps, 5 * fs, 5 * ps, seg, 5, layout, xy, al, k, lkp, dst, st)
    timings["lk"] = _compare({"%d/%d" % (x, g): dataclasses.replace(base, xcd_pyramid=best_pyr, xcd_lk=x, lk_ppg=g)
                              for x in XCD_CANDIDATES for g in LK_PPG_CANDIDATES}, step or lk_fn, reps, rounds)
    best_lk = _pick(timings["lk"], "%d/%d" % (base.xcd_lk, base.lk_ppg))
    xl, gl = (int(v) for v in best_lk.split("/"))

    # warp: a small similarity per frame
    th = torch.linspace(-0.01, 0.01, n, dtype=torch.float64, device=frames.device)
    cx, cy = (w - 1) / 2, (h - 1) / 2
    a, b = torch.cos(th) * 1.002, torch.sin(th) * 1.002
    mats = torch.stack([a, -b, cx - a * cx + b * cy + 1.5, b, a, cy - b * cx - a * cy - 0.75], 1).contiguous()
    out = torch.empty_like(frames)
    warp_fn = lambda: V.vs_warp_frame(frames, fs, w, h, w, mats, 6, out, fs, w, n, 0)
    timings["warp"] = _compare({str(x): dataclasses.replace(base, xcd_pyramid=best_pyr, xcd_lk=xl, lk_ppg=gl, xcd_warp=x)
                                for x in XCD_CANDIDATES}, step or warp_fn, reps, rounds)
    best_warp = int(_pick(timings["warp"], str(base.xcd_warp)))
    cur = Tuning(best_pyr, xl, best_warp, gl)

    # corner response: wave segment height
    det_fn = lambda: V.vs_detect_corners(frames, 5 * fs, w, h, w, seg, 5, None, 0, dp, k, xy, None, cnt, al, ws, wsb)
    timings["detect"] = _compare({str(r): dataclasses.replace(cur, det_rows=r) for r in DET_ROWS_CANDIDATES},
                                 step or det_fn, reps, rounds)
    cur = dataclasses.replace(cur, det_rows=int(_pick(timings["detect"], str(base.det_rows))))

    # fit: hypothesis workgroups in flight, on the pairs tracked above
    set_tuning(cur)
    lk_fn()
    fp = V.vs_fit_params(V.VS_HYBRID, 128, 1.0, 1, 0, 10, 20, cx, cy)
    fstate = torch.zeros(V.FIT_STATE_BYTES, dtype=torch.uint8, device=frames.device)
    prm = torch.zeros((seg, 4), dtype=torch.float64, device=frames.device)
    info = torch.zeros(seg * V.FIT_INFO_BYTES, dtype=torch.uint8, device=frames.device)
    fwsb = V.vs_fit_workspace(seg, k)
    fws = torch.empty(fwsb, dtype=torch.uint8, device=frames.device)
    # the tracked pairs sit at every 5th record: their points as consecutive items
    src5, dst5, st5 = (t[0::5][:seg].contiguous() for t in (xy, dst, st))

    def fit_fn():
        V.vs_fit_state_init(fstate)
        V.vs_fit_similarity(src5, dst5, st5, k, seg, fp, 0, fstate, prm, info, None, fws, fwsb)
    timings["fit"] = _compare({str(g): dataclasses.replace(cur, fit_groups=g) for g in FIT_GROUPS_CANDIDATES},
                              step or fit_fn, reps, rounds)
    cur = dataclasses.replace(cur, fit_groups=int(_pick(timings["fit"], str(base.fit_groups))))

    t = cur
    set_tuning(t)
    if save:
        store(cache_key(device_arch(frames.device.index or 0), w, h, k), t, timings,
              {"frames": n, "width": w, "height": h, "k": k, "levels": levels}, path)
    return t, timings
