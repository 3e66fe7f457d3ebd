"""CPU oracle of the stabilization hot path (arXiv 1701.03572), ctypes front end of vs_oracle.c.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the CPU-baseline leg of the
benchmark, never by the product path. It does not import the HIP package, and the HIP package
does not import it.

Every function takes plain numpy arrays; floating point is binary64. ``stabilize`` chains the
steps in the order of the paper's motion-estimation workflow (Section 4.1, last paragraph):
detect corners, track them by optical flow, weed by the backward check, skip the frame if too few
points remain, decide the model once per dwell block, store the parameters; then smooth the
trajectory (Section 5.1) and warp every frame (Section 5).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vs_oracle.c")
_LIB = os.path.join(_HERE, "libvs_oracle.so")
_lib = None

RIGID, SIMILARITY, HYBRID, AFFINE, HYBRID3 = 0, 1, 2, 3, 4


def build(force: bool = False) -> str:
    """Compile vs_oracle.c with gcc (binary64, no contraction, no fast-math, one thread)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-shared", "-fPIC",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class LKParams(C.Structure):
    _fields_ = [("win_half", C.c_int), ("max_iter", C.c_int), ("eps", C.c_double), ("min_eig", C.c_double),
                ("fb", C.c_int), ("fb_thresh", C.c_double)]


class FitParams(C.Structure):
    _fields_ = [("model", C.c_int32), ("ransac_iters", C.c_int32), ("inlier_thresh", C.c_double),
                ("seed", C.c_uint64), ("stream_id", C.c_int64), ("min_valid", C.c_int32), ("dwell", C.c_int32),
                ("cx", C.c_double), ("cy", C.c_double)]


class HybridState(C.Structure):
    _fields_ = [("block", C.c_int64), ("model", C.c_int32), ("decided", C.c_int32)]


class FitInfo(C.Structure):
    _fields_ = [("model", C.c_int32), ("n_valid", C.c_int32), ("n_inliers", C.c_int32), ("skipped", C.c_int32),
                ("decided_here", C.c_int32), ("pad", C.c_int32), ("err_rigid", C.c_double),
                ("err_sim", C.c_double), ("err_affine", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad"}


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        P = C.c_void_p
        _lib.vso_pyr_down.argtypes = [P, C.c_int, C.c_int, C.c_int, P, C.c_int]
        _lib.vso_min_eig_map.argtypes = [P, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, P]
        _lib.vso_tensor_map.argtypes = [P, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, P]
        _lib.vso_greedy_select.argtypes = [P, P, C.c_int, C.c_int, C.c_int, P]
        _lib.vso_greedy_select.restype = C.c_int
        _lib.vso_detect.argtypes = [P, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double, C.c_int, C.c_int, C.c_int,
                                    P, P, P]
        _lib.vso_detect.restype = C.c_int
        _lib.vso_track_lk.argtypes = [P, P, P, P, P, C.c_int, P, C.c_int, P, C.POINTER(LKParams), P, P, P, P, P]
        _lib.vso_draw.argtypes = [C.c_uint64, C.c_int64, C.c_int64, C.c_int, C.c_int]
        _lib.vso_draw.restype = C.c_uint64
        _lib.vso_draw3.argtypes = [C.c_uint64, C.c_int64, C.c_int64, C.c_int, C.c_int]
        _lib.vso_draw3.restype = C.c_uint64
        _lib.vso_fit_pair.argtypes = [P, P, P, C.c_int, C.POINTER(FitParams), C.c_int64, C.POINTER(HybridState), P,
                                      P, C.POINTER(FitInfo), P]
        _lib.vso_smooth.argtypes = [P, C.c_int, C.c_int, C.c_int, C.c_double, C.c_double, C.c_double, C.c_double,
                                    P, P, P]
        _lib.vso_warp.argtypes = [P, C.c_int, C.c_int, C.c_int, P, P, C.c_int, C.c_int]
        _lib.vso_photo_global.argtypes = [P, P, C.c_int, C.c_int, C.c_int, P, C.c_double, C.c_double, C.c_double,
                                          C.c_int, C.c_int, C.c_int, C.c_int, P]
        _lib.vso_photo_feature.argtypes = [P, P, C.c_int, C.c_int, C.c_int, P, P, C.c_int, C.c_int, P, P]
        _lib.vso_photo_refine.argtypes = [P, P, C.c_int, C.c_int, C.c_int, P, C.c_double, C.c_double, C.c_double,
                                          C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, P, P]
        _lib.vso_photo_refine.restype = C.c_int
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _u8(a):
    return np.ascontiguousarray(a, dtype=np.uint8)


# ---------------------------------------------------------------------------------------------
# O-1 pyramid
# ---------------------------------------------------------------------------------------------

def pyr_down(img: np.ndarray) -> np.ndarray:
    img = _u8(img)
    h, w = img.shape
    out = np.empty(((h + 1) // 2, (w + 1) // 2), np.uint8)
    lib().vso_pyr_down(_p(img), w, h, w, _p(out), out.shape[1])
    return out


def pyramid(img: np.ndarray, levels: int) -> list:
    out = [_u8(img)]
    for _ in range(1, levels):
        out.append(pyr_down(out[-1]))
    return out


# ---------------------------------------------------------------------------------------------
# O-2 corners
# ---------------------------------------------------------------------------------------------

def roi_margins(w: int, h: int) -> tuple:
    return max(16, w // 20), max(16, h // 20)


def min_eig_map(img: np.ndarray, rect) -> np.ndarray:
    img = _u8(img)
    h, w = img.shape
    x0, y0, x1, y1 = rect
    out = np.empty((y1 - y0, x1 - x0), np.float64)
    lib().vso_min_eig_map(_p(img), w, h, w, x0, y0, x1, y1, _p(out))
    return out


def tensor_map(img: np.ndarray, rect) -> np.ndarray:
    img = _u8(img)
    h, w = img.shape
    x0, y0, x1, y1 = rect
    out = np.empty((y1 - y0, x1 - x0, 3), np.int64)
    lib().vso_tensor_map(_p(img), w, h, w, x0, y0, x1, y1, _p(out))
    return out


def greedy_select(xs, ys, K: int, min_dist: int) -> np.ndarray:
    xs = np.ascontiguousarray(xs, np.int32)
    ys = np.ascontiguousarray(ys, np.int32)
    acc = np.empty(K + 1, np.int32)
    na = lib().vso_greedy_select(_p(xs), _p(ys), len(xs), K, min_dist, _p(acc))
    return acc[:na].copy()


def detect(img: np.ndarray, K: int, quality: float = 0.01, min_dist: int = 10, roi=None):
    """Returns (xy [k,2] float64, score [k] float64, n_candidates)."""
    img = _u8(img)
    h, w = img.shape
    mx, my = roi if roi is not None else roi_margins(w, h)
    xy = np.empty((max(K, 1), 2), np.float64)
    sc = np.empty(max(K, 1), np.float64)
    nc = C.c_int(0)
    n = lib().vso_detect(_p(img), w, h, w, K, quality, min_dist, mx, my, _p(xy), _p(sc), C.byref(nc))
    return xy[:n].copy(), sc[:n].copy(), nc.value


# ---------------------------------------------------------------------------------------------
# O-3 Lucas-Kanade
# ---------------------------------------------------------------------------------------------

def track_lk(prev_pyr: list, next_pyr: list, pts: np.ndarray, alive=None, win_half=10, max_iter=30, eps=1e-3,
             min_eig=1e-2, fb=True, fb_thresh=1.0, with_margin: bool = False):
    """Returns (xy_next [n,2], status [n] uint8, fb_err [n], iters [n,2]), plus eig_margin [n] when
    ``with_margin``: the smallest |lambda_min / window size - min_eig| / min_eig over every level of
    both passes (how close the point came to the eigenvalue test's threshold)."""
    L = len(prev_pyr)
    pv = [_u8(a) for a in prev_pyr]
    nx = [_u8(a) for a in next_pyr]
    lw = np.array([a.shape[1] for a in pv], np.int32)
    lh = np.array([a.shape[0] for a in pv], np.int32)
    pp = (C.c_void_p * L)(*[a.ctypes.data for a in pv])
    npp = (C.c_void_p * L)(*[a.ctypes.data for a in nx])
    pts = np.ascontiguousarray(pts, np.float64).reshape(-1, 2)
    n = len(pts)
    al = None if alive is None else np.ascontiguousarray(alive, np.uint8)
    prm = LKParams(win_half, max_iter, eps, min_eig, int(fb), fb_thresh)
    out = np.empty((n, 2), np.float64)
    st = np.empty(n, np.uint8)
    fe = np.empty(n, np.float64)
    it = np.empty((n, 2), np.int32)
    mg = np.empty(n, np.float64)
    lib().vso_track_lk(pp, npp, _p(lw), _p(lh), _p(lw), L, _p(pts), n, None if al is None else _p(al),
                       C.byref(prm), _p(out), _p(st), _p(fe), _p(it), _p(mg))
    if with_margin:
        return out, st, fe, it, mg
    return out, st, fe, it


# ---------------------------------------------------------------------------------------------
# O-4 robust fit
# ---------------------------------------------------------------------------------------------

def draw(seed: int, stream_id: int, pair_index: int, h: int, k: int) -> int:
    return int(lib().vso_draw(seed, stream_id, pair_index, h, k))


def fit_params(model, ransac_iters, inlier_thresh, seed, stream_id, min_valid, dwell, w, h) -> FitParams:
    return FitParams(model, ransac_iters, inlier_thresh, seed, stream_id, min_valid, dwell, (w - 1) / 2.0,
                     (h - 1) / 2.0)


def new_hybrid_state() -> HybridState:
    return HybridState(-1, SIMILARITY, 0)


def draw3(seed: int, stream_id: int, pair_index: int, h: int, k: int) -> int:
    return int(lib().vso_draw3(seed, stream_id, pair_index, h, k))


def fit_pair_affine(src, dst, valid, fp: FitParams, pair_index: int, state: HybridState | None = None):
    """Returns (params4 (a, b, tx, ty) centred, affine6 (a11, a12, tx, a21, a22, ty) centred, info
    dict, inlier flags per slot). For an affine result params4 is its nearest similarity."""
    src = np.ascontiguousarray(src, np.float64).reshape(-1, 2)
    dst = np.ascontiguousarray(dst, np.float64).reshape(-1, 2)
    n = len(src)
    v = None if valid is None else np.ascontiguousarray(valid, np.uint8)
    st = state if state is not None else new_hybrid_state()
    out = np.empty(4, np.float64)
    m6 = np.empty(6, np.float64)
    info = FitInfo()
    inl = np.empty(max(n, 1), np.uint8)
    lib().vso_fit_pair(_p(src), _p(dst), None if v is None else _p(v), n, C.byref(fp), pair_index, C.byref(st),
                       _p(out), _p(m6), C.byref(info), _p(inl))
    return out, m6, info.as_dict(), inl[:n].copy()


def fit_pair(src, dst, valid, fp: FitParams, pair_index: int, state: HybridState | None = None):
    """Returns (params4 (a, b, tx, ty) centred, info dict, inlier flags per slot)."""
    out, _, info, inl = fit_pair_affine(src, dst, valid, fp, pair_index, state)
    return out, info, inl


# ---------------------------------------------------------------------------------------------
# O-5 smoothing
# ---------------------------------------------------------------------------------------------

def smooth(pair_params: np.ndarray, n_frames: int, mode: int, radius: int, ratio: float, crop: float, w: int,
           h: int):
    """Returns (traj [n,4], smoothed [n,4], mats [n,6] src->dst pixel coordinates)."""
    pp = np.ascontiguousarray(pair_params, np.float64).reshape(-1, 4)
    assert len(pp) == max(n_frames - 1, 0)
    traj = np.empty((n_frames, 4))
    sm = np.empty((n_frames, 4))
    mats = np.empty((n_frames, 6))
    lib().vso_smooth(_p(pp) if len(pp) else None, n_frames, mode, radius, ratio, crop, (w - 1) / 2.0,
                     (h - 1) / 2.0, _p(traj), _p(sm), _p(mats))
    return traj, sm, mats


# ---------------------------------------------------------------------------------------------
# O-6 warp
# ---------------------------------------------------------------------------------------------

def warp(img: np.ndarray, M, border: int = 0) -> np.ndarray:
    img = _u8(img)
    h, w = img.shape
    M = np.ascontiguousarray(M, np.float64).reshape(6)
    out = np.empty_like(img)
    lib().vso_warp(_p(img), w, h, w, _p(M), _p(out), w, border)
    return out


# ---------------------------------------------------------------------------------------------
# O-7 photometric loss, gradient and Gauss-Newton refinement (project extension)
# ---------------------------------------------------------------------------------------------

def photo_frame(w: int, h: int) -> tuple:
    """Centre c = ((W-1)/2, (H-1)/2) and scale rho = max(W, H) / 2 of the transform parameters."""
    return (w - 1) / 2.0, (h - 1) / 2.0, max(w, h) / 2.0


def theta_from_fit(params4, w: int, h: int) -> np.ndarray:
    """theta of the fitted similarity (a, b, tx, ty) in centred coordinates: (rho (a - 1), rho b, tx, ty)."""
    a, b, tx, ty = (float(v) for v in params4)
    rho = photo_frame(w, h)[2]
    return np.array([rho * (a - 1.0), rho * b, tx, ty])


def photo_omega(theta, w: int, h: int, extra: int = 0) -> tuple:
    """Inner rectangle (x0, y0, x1, y1) whose margin is ceil(max |T(x) - x|) + 2 + extra over the
    frame corners (for this transform the displacement is largest at a corner)."""
    cx, cy, rho = photo_frame(w, h)
    th = np.asarray(theta, np.float64)
    best = 0.0
    for x in (0, w - 1):
        for y in (0, h - 1):
            dx, dy = (x - cx) / rho, (y - cy) / rho
            mx = th[0] * dx - th[1] * dy + th[2]
            my = th[1] * dx + th[0] * dy + th[3]
            best = max(best, float(np.hypot(mx, my)))
    m = int(np.ceil(best)) + 2 + extra
    return m, m, w - m, h - m


def photo_global(f0: np.ndarray, f1: np.ndarray, theta, omega) -> dict:
    """Global loss, dL/dtheta, J^T J (4x4) and J^T r over the rectangle omega."""
    f0, f1 = _u8(f0), _u8(f1)
    h, w = f0.shape
    cx, cy, rho = photo_frame(w, h)
    th = np.ascontiguousarray(theta, np.float64)
    out = np.zeros(19)
    lib().vso_photo_global(_p(f0), _p(f1), w, h, w, _p(th), cx, cy, rho, *[int(v) for v in omega], _p(out))
    jtj = np.zeros((4, 4))
    t = 5
    for i in range(4):
        for j in range(i, 4):
            jtj[i, j] = jtj[j, i] = out[t]
            t += 1
    return {"loss": out[0], "grad": out[1:5].copy(), "jtj": jtj, "jtr": out[15:19].copy()}


def photo_feature(f0: np.ndarray, f1: np.ndarray, u, d, win_half: int = 10):
    """Per-point window loss and its gradient with respect to the displacement d."""
    f0, f1 = _u8(f0), _u8(f1)
    h, w = f0.shape
    u = np.ascontiguousarray(u, np.float64).reshape(-1, 2)
    d = np.ascontiguousarray(d, np.float64).reshape(-1, 2)
    m = len(u)
    loss, grad = np.zeros(m), np.zeros((m, 2))
    lib().vso_photo_feature(_p(f0), _p(f1), w, h, w, _p(u), _p(d), m, win_half, _p(loss), _p(grad))
    return loss, grad


def photo_refine(f0: np.ndarray, f1: np.ndarray, theta0, omega, max_steps: int = 5):
    """Gauss-Newton refinement; returns (theta, (initial loss, final loss), accepted steps)."""
    f0, f1 = _u8(f0), _u8(f1)
    h, w = f0.shape
    cx, cy, rho = photo_frame(w, h)
    th0 = np.ascontiguousarray(theta0, np.float64)
    th, lo = np.zeros(4), np.zeros(2)
    k = lib().vso_photo_refine(_p(f0), _p(f1), w, h, w, _p(th0), cx, cy, rho, *[int(v) for v in omega], max_steps,
                               _p(th), _p(lo))
    return th, (lo[0], lo[1]), int(k)


# ---------------------------------------------------------------------------------------------
# whole sequence
# ---------------------------------------------------------------------------------------------

def _segment_tracks(frames: np.ndarray, P, roi, first: int, last: int) -> list:
    """Detection and tracking of frames first..last (first a re-detection frame, last the next one or
    the final frame): detect on ``first``, track pair by pair, chain the tracked points, and re-detect
    after a pair with fewer than min_valid valid points (the fit skips such a pair). Returns one
    record per pair plus the detections made, exactly as the whole-sequence loop makes them."""
    recs = []
    pyr_prev = pyramid(frames[first], P.levels)
    pts, _, _ = detect(frames[first], P.max_corners, P.quality, P.min_dist, roi)
    alive = np.ones(len(pts), np.uint8)
    dets = {first: pts.copy()}
    for j in range(first + 1, last + 1):
        pyr_next = pyramid(frames[j], P.levels)
        nxt, status, fb_err, iters = track_lk(pyr_prev, pyr_next, pts, alive, P.win_half, P.max_iter, P.eps,
                                              P.min_eig, P.fb, P.fb_thresh)
        recs.append({"src": pts.copy(), "dst": nxt, "status": status, "fb_err": fb_err, "iters": iters})
        if j == last:
            break
        if j % P.redetect_every == 0 or int(status.sum()) < P.min_valid:
            pts, _, _ = detect(frames[j], P.max_corners, P.quality, P.min_dist, roi)
            alive = np.ones(len(pts), np.uint8)
            dets[j] = pts.copy()
        else:
            pts, alive = nxt, status
        pyr_prev = pyr_next
    return recs, dets


def stabilize(frames: np.ndarray, P, warp_frames: bool = True, max_pairs: int | None = None, workers: int = 1) -> dict:
    """Run the whole path on uint8 frames [n, H, W] with parameters ``P`` (attributes as in the
    package's StabParams; read by name only). Returns every intermediate the tests compare.

    workers > 1 runs the detection and tracking of the re-detection segments in that many threads
    (the C calls release the interpreter lock) and the warps likewise; the fits, the refinement and the
    smoothing stay in pair order. Segments are independent: every segment starts from a fresh
    detection, and a skipped pair (fewer than min_valid valid points) forces a re-detection inside its
    own segment, decided by the tracking alone. The results are identical to workers = 1 (tested)."""
    if workers > 1:
        return _stabilize_threaded(frames, P, warp_frames, max_pairs, workers)
    n, H, W = frames.shape
    n_pairs = n - 1 if max_pairs is None else min(n - 1, max_pairs)
    n_used = n_pairs + 1
    roi = (P.roi_mx if P.roi_mx is not None else max(16, W // 20),
           P.roi_my if P.roi_my is not None else max(16, H // 20))
    fp = fit_params(P.model, P.ransac_iters, P.inlier_thresh, P.seed, P.stream_id, P.min_valid, P.dwell, W, H)
    st = new_hybrid_state()
    pyr_prev = pyramid(frames[0], P.levels)
    pts, _, _ = detect(frames[0], P.max_corners, P.quality, P.min_dist, roi)
    alive = np.ones(len(pts), np.uint8)
    detect_frames = [0]
    out = {"pair_params": np.zeros((n_pairs, 4)), "info": [], "tracks": [], "detections": {0: pts.copy()}}
    for j in range(1, n_used):
        pyr_next = pyramid(frames[j], P.levels)
        nxt, status, fb_err, iters = track_lk(pyr_prev, pyr_next, pts, alive, P.win_half, P.max_iter, P.eps,
                                              P.min_eig, P.fb, P.fb_thresh)
        prm, info, inl = fit_pair(pts, nxt, status, fp, j - 1, st)
        prm = _refined(frames, P, j, prm, info, W, H)
        out["pair_params"][j - 1] = prm
        out["info"].append(info)
        out["tracks"].append({"src": pts.copy(), "dst": nxt, "status": status, "fb_err": fb_err, "iters": iters,
                              "inliers": inl})
        if j % P.redetect_every == 0 or info["skipped"]:
            pts, _, _ = detect(frames[j], P.max_corners, P.quality, P.min_dist, roi)
            alive = np.ones(len(pts), np.uint8)
            detect_frames.append(j)
            out["detections"][j] = pts.copy()
        else:
            pts, alive = nxt, status
        pyr_prev = pyr_next
    traj, sm, mats = smooth(out["pair_params"], n_used, P.smooth_mode, P.radius, P.kalman_ratio, P.crop, W, H)
    out.update(traj=traj, smoothed=sm, mats=mats, detect_frames=detect_frames)
    if warp_frames:
        out["warped"] = np.stack([warp(frames[j], mats[j], P.border) for j in range(n_used)])
    return out


def _refined(frames, P, j, prm, info, W, H):
    """Optional photometric refinement of the fitted similarity of pair j-1 -> j (O-7), in its
    (a, b, tx, ty) form; skipped pairs stay as they are."""
    steps = getattr(P, "photometric_steps", 0)
    if steps <= 0 or info["skipped"]:
        return prm
    m = P.photometric_margin if getattr(P, "photometric_margin", None) is not None else max(16, min(W, H) // 10)
    th, _, _ = photo_refine(frames[j - 1], frames[j], theta_from_fit(prm, W, H), (m, m, W - m, H - m), steps)
    rho = photo_frame(W, H)[2]
    return np.array([1.0 + th[0] / rho, th[1] / rho, th[2], th[3]])


def _stabilize_threaded(frames, P, warp_frames, max_pairs, workers):
    import concurrent.futures as cf
    n, H, W = frames.shape
    n_pairs = n - 1 if max_pairs is None else min(n - 1, max_pairs)
    n_used = n_pairs + 1
    roi = (P.roi_mx if P.roi_mx is not None else max(16, W // 20),
           P.roi_my if P.roi_my is not None else max(16, H // 20))
    e = P.redetect_every
    segs = [(s, min(s + e, n_used - 1)) for s in range(0, n_used - 1, e)]
    lib()
    with cf.ThreadPoolExecutor(workers) as ex:
        parts = list(ex.map(lambda fl: _segment_tracks(frames, P, roi, fl[0], fl[1]), segs))
    fp = fit_params(P.model, P.ransac_iters, P.inlier_thresh, P.seed, P.stream_id, P.min_valid, P.dwell, W, H)
    st = new_hybrid_state()
    out = {"pair_params": np.zeros((n_pairs, 4)), "info": [], "tracks": [], "detections": {}}
    if n_pairs == 0:
        pts, _, _ = detect(frames[0], P.max_corners, P.quality, P.min_dist, roi)
        out["detections"][0] = pts
    detect_frames = []
    for recs, dets in parts:
        out["detections"].update(dets)
        detect_frames += sorted(dets)
        out["tracks"] += recs
    for k, t in enumerate(out["tracks"]):
        prm, info, inl = fit_pair(t["src"], t["dst"], t["status"], fp, k, st)
        out["pair_params"][k] = _refined(frames, P, k + 1, prm, info, W, H)
        out["info"].append(info)
        t["inliers"] = inl
    traj, sm, mats = smooth(out["pair_params"], n_used, P.smooth_mode, P.radius, P.kalman_ratio, P.crop, W, H)
    out.update(traj=traj, smoothed=sm, mats=mats, detect_frames=detect_frames if n_pairs else [0])
    if warp_frames:
        with cf.ThreadPoolExecutor(workers) as ex:
            out["warped"] = np.stack(list(ex.map(lambda j: warp(frames[j], mats[j], P.border), range(n_used))))
    return out
