"""Thin Python binding of libvstab (include/vstab.h): argument marshalling only.

Every function has the name of its C entry point and takes device tensors (torch, on the GPU) or
raw integer device addresses; every operation runs in the library's HIP kernels on the caller's
current torch stream. Errors raise ``VsError`` with the library's message. Loading fails loudly
when the library is missing: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvstab.so")

VS_MAX_LEVELS = 8
VS_MAX_CORNERS = 4096
VS_TRAJ_RING = 256
VS_FIT_NOALLOC_SCRATCH_BYTES = 8 * 1024 * 1024
VS_RIGID, VS_SIMILARITY, VS_HYBRID, VS_AFFINE, VS_HYBRID3 = 0, 1, 2, 3, 4
VS_SMOOTH_CENTERED, VS_SMOOTH_CAUSAL, VS_SMOOTH_KALMAN = 0, 1, 2


class VsError(RuntimeError):
    pass


class vs_tuning(C.Structure):
    _fields_ = [("xcd_min_items_pyramid", C.c_int32), ("xcd_min_items_lk", C.c_int32),
                ("xcd_min_items_warp", C.c_int32), ("lk_points_per_group", C.c_int32),
                ("detect_segment_rows", C.c_int32), ("fit_groups_in_flight", C.c_int32)]


class vs_pyramid(C.Structure):
    _fields_ = [("levels", C.c_int32), ("width", C.c_int32 * VS_MAX_LEVELS), ("height", C.c_int32 * VS_MAX_LEVELS),
                ("pitch", C.c_int32 * VS_MAX_LEVELS), ("offset", C.c_int64 * VS_MAX_LEVELS), ("bytes", C.c_int64)]


class vs_detect_params(C.Structure):
    _fields_ = [("max_corners", C.c_int32), ("quality", C.c_double), ("min_dist", C.c_int32),
                ("roi_mx", C.c_int32), ("roi_my", C.c_int32), ("max_corners_per_item", C.c_void_p)]


class vs_lk_params(C.Structure):
    _fields_ = [("win_half", C.c_int32), ("max_iter", C.c_int32), ("eps", C.c_float), ("min_eig", C.c_float),
                ("fb", C.c_int32), ("fb_thresh", C.c_float)]


class vs_fit_params(C.Structure):
    _fields_ = [("model", C.c_int32), ("ransac_iters", C.c_int32), ("inlier_thresh", C.c_double),
                ("seed", C.c_uint64), ("stream_id", C.c_int64), ("min_valid", C.c_int32), ("dwell", C.c_int32),
                ("cx", C.c_double), ("cy", C.c_double)]


class vs_fit_state(C.Structure):
    _fields_ = [("block", C.c_int64), ("model", C.c_int32), ("decided", C.c_int32)]


class vs_fit_info(C.Structure):
    _fields_ = [("model", C.c_int32), ("n_valid", C.c_int32), ("n_inliers", C.c_int32), ("skipped", C.c_int32),
                ("decided_here", C.c_int32), ("pad", C.c_int32), ("err_rigid", C.c_double), ("err_sim", C.c_double),
                ("err_affine", C.c_double)]


class vs_rect(C.Structure):
    _fields_ = [("x0", C.c_int32), ("y0", C.c_int32), ("x1", C.c_int32), ("y1", C.c_int32)]


VS_PHOTO_SUMS = 19


class vs_smooth_params(C.Structure):
    _fields_ = [("mode", C.c_int32), ("radius", C.c_int32), ("kalman_ratio", C.c_double), ("crop", C.c_double),
                ("cx", C.c_double), ("cy", C.c_double)]


VS_STREAM_MAX_FRAMES = 160


class vs_stream(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("layout", vs_pyramid), ("detect", vs_detect_params),
                ("lk", vs_lk_params), ("fit", vs_fit_params), ("smooth", vs_smooth_params), ("capacity", C.c_int32),
                ("redetect_every", C.c_int32), ("min_valid", C.c_int32), ("border", C.c_int32),
                ("out_slots", C.c_int32), ("photo_steps", C.c_int32), ("photo_omega", vs_rect),
                ("pyr", C.c_void_p), ("pts", C.c_void_p), ("alive", C.c_void_p), ("dst", C.c_void_p),
                ("status", C.c_void_p), ("fb_err", C.c_void_p), ("n_valid", C.c_void_p), ("count", C.c_void_p),
                ("detect_ws", C.c_void_p), ("detect_ws_bytes", C.c_size_t), ("fit_ws", C.c_void_p),
                ("fit_ws_bytes", C.c_size_t), ("fit_state", C.c_void_p), ("pair_params", C.c_void_p),
                ("affine6", C.c_void_p), ("info", C.c_void_p), ("inliers", C.c_void_p), ("traj_state", C.c_void_p),
                ("mats", C.c_void_p), ("n_emitted", C.c_void_p), ("first_frame", C.c_void_p),
                ("photo_loss", C.c_void_p), ("photo_accepted", C.c_void_p), ("photo_ws", C.c_void_p),
                ("photo_ws_bytes", C.c_size_t), ("out", C.c_void_p), ("ready_event", C.c_void_p), ("ring", C.c_void_p),
                ("ring_len", C.c_int32), ("ring_pad", C.c_int32), ("next_frame", C.c_int64),
                ("emitted", C.c_int64), ("frames", C.c_void_p * VS_STREAM_MAX_FRAMES)]


VS_BATCH_MAX_STREAMS = 256


class vs_batch(C.Structure):
    _fields_ = [("proto", vs_stream), ("max_streams", C.c_int32), ("detect_chunk", C.c_int32),
                ("workspace", C.c_void_p), ("ws_bytes", C.c_size_t), ("ready_event", C.c_void_p),
                ("attached", C.c_void_p * VS_BATCH_MAX_STREAMS)]


FIT_INFO_BYTES = C.sizeof(vs_fit_info)
FIT_INFO_SKIPPED_OFFSET = vs_fit_info.skipped.offset
FIT_STATE_BYTES = C.sizeof(vs_fit_state)

# numpy/torch view of vs_fit_info records
FIT_INFO_FIELDS = [n for n, _ in vs_fit_info._fields_]

_P = C.c_void_p
_SIGS = {
    "vs_pyramid_layout": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.POINTER(vs_pyramid)]),
    "vs_build_pyramid": (C.c_int, [_P, C.c_int64, _P, C.c_int64, C.c_int32, C.POINTER(vs_pyramid), _P]),
    "vs_detect_workspace": (C.c_size_t, [C.c_int32, C.c_int32, C.c_int32]),
    "vs_detect_corners": (C.c_int, [_P, C.c_int64, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32, _P, C.c_int32,
                                    C.POINTER(vs_detect_params), C.c_int32, _P, _P, _P, _P, _P, C.c_size_t, _P]),
    "vs_track_lk": (C.c_int, [_P, _P, _P, _P, C.c_int64, C.c_int64, C.c_int32, C.c_int32, C.POINTER(vs_pyramid), _P, _P,
                              C.c_int32, C.POINTER(vs_lk_params), _P, _P, _P, _P, _P, _P, _P, _P]),
    "vs_track_lk_segments": (C.c_int, [_P, _P, C.c_int64, C.c_int64, C.c_int64, C.c_int64, C.c_int32, C.c_int32,
                                       C.c_int32, C.c_int32, C.c_int32, C.POINTER(vs_pyramid), C.c_int32,
                                       C.POINTER(vs_lk_params), _P, _P, _P, _P, _P, _P, _P, C.c_int32, _P, _P]),
    "vs_fit_workspace": (C.c_size_t, [C.c_int32, C.c_int32]),
    "vs_fit_state_init": (C.c_int, [_P, _P]),
    "vs_fit_similarity": (C.c_int, [_P, _P, _P, C.c_int32, C.c_int32, C.POINTER(vs_fit_params), C.c_int64, _P, _P,
                                    _P, _P, _P, C.c_size_t, _P]),
    "vs_fit_motion": (C.c_int, [_P, _P, _P, C.c_int32, C.c_int32, C.POINTER(vs_fit_params), C.c_int64, _P, _P, _P,
                                _P, _P, _P, C.c_size_t, _P]),
    "vs_fit_noalloc_max_pairs": (C.c_int32, [C.c_int32]),
    "vs_fit_motion_noalloc": (C.c_int, [_P, _P, _P, C.c_int32, C.c_int32, C.POINTER(vs_fit_params), C.c_int64, _P,
                                        _P, _P, _P, _P, _P]),
    "vs_traj_state_bytes": (C.c_size_t, []),
    "vs_traj_state_init": (C.c_int, [_P, _P]),
    "vs_smooth_trajectory": (C.c_int, [_P, C.c_int32, C.c_int32, C.POINTER(vs_smooth_params), _P, _P, C.c_int32,
                                       _P, _P, _P]),
    "vs_warp_frame": (C.c_int, [_P, C.c_int64, C.c_int32, C.c_int32, C.c_int32, _P, C.c_int64, _P, C.c_int64,
                                C.c_int32, C.c_int32, C.c_int32, _P]),
    "vs_photometric_fwd": (C.c_int, [_P, _P, C.c_int64, C.c_int32, C.c_int32, C.c_int32, C.c_int32, _P, C.c_int64,
                                     C.c_double, C.c_double, C.c_double, C.POINTER(vs_rect), _P, _P, C.c_size_t, _P]),
    "vs_photometric_bwd": (C.c_int, [_P, _P, C.c_int64, C.c_int32, C.c_int32, C.c_int32, C.c_int32, _P, C.c_int64,
                                     C.c_double, C.c_double, C.c_double, C.POINTER(vs_rect), _P, _P, C.c_size_t, _P]),
    "vs_photometric_features": (C.c_int, [_P, _P, C.c_int64, C.c_int32, C.c_int32, C.c_int32, C.c_int32, _P, _P,
                                          C.c_int32, C.c_int32, _P, _P, _P]),
    "vs_photometric_workspace": (C.c_size_t, [C.c_int32, C.c_int32, C.c_int32]),
    "vs_photometric_refine": (C.c_int, [_P, _P, C.c_int64, C.c_int32, C.c_int32, C.c_int32, C.c_int32, _P, _P,
                                        C.c_int64, C.c_int32, _P, C.c_int64, C.c_double, C.c_double, C.c_double,
                                        C.POINTER(vs_rect), C.c_int32, _P, _P, _P, C.c_size_t, _P]),
    "vs_stream_reset": (C.c_int, [C.POINTER(vs_stream), _P]),
    "vs_stream_push": (C.c_int, [C.POINTER(vs_stream), _P, C.POINTER(C.c_int64), C.POINTER(C.c_int32), _P]),
    "vs_stream_flush": (C.c_int, [C.POINTER(vs_stream), C.POINTER(C.c_int64), C.POINTER(C.c_int32), _P]),
    "vs_batch_workspace": (C.c_size_t, [C.POINTER(vs_stream), C.c_int32, C.c_int32]),
    "vs_batch_init": (C.c_int, [C.POINTER(vs_batch), C.POINTER(vs_stream), C.c_int32, C.c_int32, _P, C.c_size_t]),
    "vs_batch_attach": (C.c_int, [C.POINTER(vs_batch), C.c_int32, C.POINTER(vs_stream), _P]),
    "vs_batch_detach": (C.c_int, [C.POINTER(vs_batch), C.c_int32]),
    "vs_batch_push": (C.c_int, [C.POINTER(vs_batch), C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int64),
                                C.POINTER(C.c_int32), _P]),
    "vs_batch_note_replayed": (C.c_int, [C.POINTER(vs_batch), C.c_int32, C.POINTER(C.c_int32), C.c_int32]),
    "vs_set_tuning": (C.c_int, [C.POINTER(vs_tuning)]),
    "vs_get_tuning": (C.c_int, [C.POINTER(vs_tuning)]),
    "vs_last_error": (C.c_char_p, []),
    "vs_version": (C.c_int, []),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load libvstab.so. Raises when it is missing: the HIP library is the only compute path."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise VsError("libvstab.so not built at %s (run __graft_entry__.build())" % path)
        lib = C.CDLL(path)
        for name, (res, args) in _SIGS.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def exported_symbols() -> list:
    return list(_SIGS)


def _ptr(x) -> int | None:
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if isinstance(x, torch.Tensor):
        if not x.is_cuda:
            raise VsError("expected a device tensor, got a %s tensor" % x.device)
        return x.data_ptr()
    raise TypeError("expected a torch device tensor or an integer address, got %r" % type(x))


def _stream(stream) -> int | None:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    return int(stream)


def _check(rc: int, what: str):
    if rc != 0:
        raise VsError("%s failed (%d): %s" % (what, rc, load().vs_last_error().decode()))


# ------------------------------------------------------------------------------------------------
# the C entry points
# ------------------------------------------------------------------------------------------------

def vs_version() -> int:
    return load().vs_version()


def vs_stream_reset(s: vs_stream, stream=None):
    _check(load().vs_stream_reset(C.byref(s), _stream(stream)), "vs_stream_reset")


def vs_stream_push(s: vs_stream, frame, stream=None) -> tuple[int, int]:
    """Returns (index of the first frame emitted by this push, number emitted)."""
    first, n = C.c_int64(0), C.c_int32(0)
    _check(load().vs_stream_push(C.byref(s), _ptr(frame), C.byref(first), C.byref(n), _stream(stream)),
           "vs_stream_push")
    return first.value, n.value


def vs_stream_flush(s: vs_stream, stream=None) -> tuple[int, int]:
    first, n = C.c_int64(0), C.c_int32(0)
    _check(load().vs_stream_flush(C.byref(s), C.byref(first), C.byref(n), _stream(stream)), "vs_stream_flush")
    return first.value, n.value


def vs_batch_workspace(proto: vs_stream, max_streams: int, detect_chunk: int) -> int:
    return int(load().vs_batch_workspace(C.byref(proto), max_streams, detect_chunk))


def vs_batch_init(b: vs_batch, proto: vs_stream, max_streams: int, detect_chunk: int, workspace, ws_bytes: int):
    _check(load().vs_batch_init(C.byref(b), C.byref(proto), max_streams, detect_chunk, _ptr(workspace), ws_bytes),
           "vs_batch_init")


def vs_batch_attach(b: vs_batch, slot: int, s: vs_stream, stream=None):
    _check(load().vs_batch_attach(C.byref(b), slot, C.byref(s), _stream(stream)), "vs_batch_attach")


def vs_batch_detach(b: vs_batch, slot: int):
    _check(load().vs_batch_detach(C.byref(b), slot), "vs_batch_detach")


def vs_batch_push(b: vs_batch, slots, stream=None) -> tuple[list, list]:
    """Returns (first emitted frame index, number emitted) per listed slot."""
    n = len(slots)
    sl = (C.c_int32 * max(n, 1))(*slots)
    first = (C.c_int64 * max(n, 1))()
    cnt = (C.c_int32 * max(n, 1))()
    _check(load().vs_batch_push(C.byref(b), n, sl, first, cnt, _stream(stream)), "vs_batch_push")
    return list(first[:n]), list(cnt[:n])


def vs_batch_note_replayed(b: vs_batch, slots, steps: int):
    n = len(slots)
    sl = (C.c_int32 * max(n, 1))(*slots)
    _check(load().vs_batch_note_replayed(C.byref(b), n, sl, steps), "vs_batch_note_replayed")


def vs_set_tuning(t: "vs_tuning | None"):
    _check(load().vs_set_tuning(None if t is None else C.byref(t)), "vs_set_tuning")


def vs_get_tuning() -> vs_tuning:
    t = vs_tuning()
    _check(load().vs_get_tuning(C.byref(t)), "vs_get_tuning")
    return t


def vs_pyramid_layout(width: int, height: int, pitch0: int, levels: int) -> vs_pyramid:
    out = vs_pyramid()
    _check(load().vs_pyramid_layout(width, height, pitch0, levels, C.byref(out)), "vs_pyramid_layout")
    return out


def vs_build_pyramid(frames, frame_stride: int, pyrs, pyr_stride: int, n: int, layout: vs_pyramid, stream=None):
    _check(load().vs_build_pyramid(_ptr(frames), frame_stride, _ptr(pyrs), pyr_stride, n, C.byref(layout),
                                   _stream(stream)), "vs_build_pyramid")


def vs_detect_workspace(width: int, height: int, n: int) -> int:
    return int(load().vs_detect_workspace(width, height, n))


def vs_detect_corners(frames, frame_stride: int, width: int, height: int, pitch: int, n: int, istride: int, gate,
                      gate_min: int, params: vs_detect_params, capacity: int, xy, score, count, alive, workspace,
                      ws_bytes: int, stream=None):
    _check(load().vs_detect_corners(_ptr(frames), frame_stride, width, height, pitch, n, istride, _ptr(gate), gate_min,
                                    C.byref(params), capacity, _ptr(xy), _ptr(score), _ptr(count), _ptr(alive),
                                    _ptr(workspace), ws_bytes, _stream(stream)), "vs_detect_corners")


def vs_track_lk(prev_frames, prev_pyrs, next_frames, next_pyrs, frame_stride: int, pyr_stride: int, n: int,
                istride: int, layout: vs_pyramid, xy_prev, alive_prev, capacity: int, params: vs_lk_params, xy_next,
                status, fb_err=None, n_valid=None, xy_chain=None, alive_chain=None, work=None, stream=None):
    _check(load().vs_track_lk(_ptr(prev_frames), _ptr(prev_pyrs), _ptr(next_frames), _ptr(next_pyrs), frame_stride,
                              pyr_stride, n, istride, C.byref(layout), _ptr(xy_prev), _ptr(alive_prev), capacity,
                              C.byref(params), _ptr(xy_next), _ptr(status), _ptr(fb_err), _ptr(n_valid),
                              _ptr(xy_chain), _ptr(alive_chain), _ptr(work), _stream(stream)), "vs_track_lk")


def vs_track_lk_segments(frames, pyrs, frame_stride: int, pyr_stride: int, frame_step: int, pyr_step: int, n: int,
                         istride: int, pairs: int, last_pairs: int, first: int, layout: vs_pyramid, capacity: int,
                         params: vs_lk_params, xy, alive, dst, status, fb_err=None, n_valid=None, gate=None,
                         gate_min: int = 0, work=None, stream=None):
    _check(load().vs_track_lk_segments(_ptr(frames), _ptr(pyrs), frame_stride, pyr_stride, frame_step, pyr_step, n,
                                       istride, pairs, last_pairs, first, C.byref(layout), capacity, C.byref(params),
                                       _ptr(xy), _ptr(alive), _ptr(dst), _ptr(status), _ptr(fb_err), _ptr(n_valid),
                                       _ptr(gate), gate_min, _ptr(work), _stream(stream)), "vs_track_lk_segments")


def vs_fit_workspace(n: int, capacity: int) -> int:
    return int(load().vs_fit_workspace(n, capacity))


def vs_fit_state_init(state, stream=None):
    _check(load().vs_fit_state_init(_ptr(state), _stream(stream)), "vs_fit_state_init")


def vs_fit_similarity(src, dst, valid, capacity: int, n: int, params: vs_fit_params, pair_index0: int, state,
                      out_params, info, inliers, workspace, ws_bytes: int, stream=None):
    _check(load().vs_fit_similarity(_ptr(src), _ptr(dst), _ptr(valid), capacity, n, C.byref(params), pair_index0,
                                    _ptr(state), _ptr(out_params), _ptr(info), _ptr(inliers), _ptr(workspace),
                                    ws_bytes, _stream(stream)), "vs_fit_similarity")


def vs_fit_motion(src, dst, valid, capacity: int, n: int, params: vs_fit_params, pair_index0: int, state,
                  out_params, affine6, info, inliers, workspace, ws_bytes: int, stream=None):
    _check(load().vs_fit_motion(_ptr(src), _ptr(dst), _ptr(valid), capacity, n, C.byref(params), pair_index0,
                                _ptr(state), _ptr(out_params), _ptr(affine6), _ptr(info), _ptr(inliers),
                                _ptr(workspace), ws_bytes, _stream(stream)), "vs_fit_motion")


def vs_fit_noalloc_max_pairs(capacity: int) -> int:
    return int(load().vs_fit_noalloc_max_pairs(capacity))


def vs_fit_motion_noalloc(src, dst, valid, capacity: int, n: int, params: vs_fit_params, pair_index0: int, state,
                          out_params, affine6, info, inliers, stream=None):
    _check(load().vs_fit_motion_noalloc(_ptr(src), _ptr(dst), _ptr(valid), capacity, n, C.byref(params), pair_index0,
                                        _ptr(state), _ptr(out_params), _ptr(affine6), _ptr(info), _ptr(inliers),
                                        _stream(stream)), "vs_fit_motion_noalloc")


def vs_traj_state_bytes() -> int:
    return int(load().vs_traj_state_bytes())


def vs_traj_state_init(state, stream=None):
    _check(load().vs_traj_state_init(_ptr(state), _stream(stream)), "vs_traj_state_init")


def vs_smooth_trajectory(pair_params, n_new: int, end_of_stream: int, params: vs_smooth_params, state, mats,
                         mats_capacity: int, n_emitted=None, first_frame=None, stream=None):
    _check(load().vs_smooth_trajectory(_ptr(pair_params), n_new, end_of_stream, C.byref(params), _ptr(state),
                                       _ptr(mats), mats_capacity, _ptr(n_emitted), _ptr(first_frame),
                                       _stream(stream)), "vs_smooth_trajectory")


def vs_warp_frame(src, src_stride: int, width: int, height: int, src_pitch: int, mats, mat_stride: int, dst,
                  dst_stride: int, dst_pitch: int, n: int, border: int = 0, stream=None):
    _check(load().vs_warp_frame(_ptr(src), src_stride, width, height, src_pitch, _ptr(mats), mat_stride, _ptr(dst),
                                dst_stride, dst_pitch, n, border, _stream(stream)), "vs_warp_frame")


def vs_photometric_fwd(prev, nxt, frame_stride: int, width: int, height: int, pitch: int, n: int, theta,
                       theta_stride: int, cx: float, cy: float, rho: float, omega: vs_rect, sums, workspace,
                       ws_bytes: int, stream=None):
    _check(load().vs_photometric_fwd(_ptr(prev), _ptr(nxt), frame_stride, width, height, pitch, n, _ptr(theta),
                                     theta_stride, cx, cy, rho, C.byref(omega), _ptr(sums), _ptr(workspace), ws_bytes,
                                     _stream(stream)), "vs_photometric_fwd")


def vs_photometric_bwd(prev, nxt, frame_stride: int, width: int, height: int, pitch: int, n: int, theta,
                       theta_stride: int, cx: float, cy: float, rho: float, omega: vs_rect, sums, workspace,
                       ws_bytes: int, stream=None):
    _check(load().vs_photometric_bwd(_ptr(prev), _ptr(nxt), frame_stride, width, height, pitch, n, _ptr(theta),
                                     theta_stride, cx, cy, rho, C.byref(omega), _ptr(sums), _ptr(workspace), ws_bytes,
                                     _stream(stream)), "vs_photometric_bwd")


def vs_photometric_features(prev, nxt, frame_stride: int, width: int, height: int, pitch: int, n: int, u, d, m: int,
                            win_half: int, loss, grad=None, stream=None):
    _check(load().vs_photometric_features(_ptr(prev), _ptr(nxt), frame_stride, width, height, pitch, n, _ptr(u),
                                          _ptr(d), m, win_half, _ptr(loss), _ptr(grad), _stream(stream)),
           "vs_photometric_features")


def vs_photometric_workspace(n: int, width: int, height: int) -> int:
    return int(load().vs_photometric_workspace(n, width, height))


VS_PHOTO_THETA, VS_PHOTO_FIT = 0, 1


def vs_photometric_refine(prev, nxt, frame_stride: int, width: int, height: int, pitch: int, n: int, theta0,
                          theta_out, theta_stride: int, param_kind: int, skip, skip_stride: int, cx: float, cy: float,
                          rho: float, omega: vs_rect, max_steps: int, loss_out, accepted, workspace, ws_bytes: int,
                          stream=None):
    _check(load().vs_photometric_refine(_ptr(prev), _ptr(nxt), frame_stride, width, height, pitch, n, _ptr(theta0),
                                        _ptr(theta_out), theta_stride, param_kind, _ptr(skip), skip_stride, cx, cy,
                                        rho, C.byref(omega), max_steps, _ptr(loss_out), _ptr(accepted),
                                        _ptr(workspace), ws_bytes, _stream(stream)), "vs_photometric_refine")


def fit_info_to_dicts(info_bytes: torch.Tensor) -> list:
    """Decode a host copy of vs_fit_info records (uint8 tensor of n * FIT_INFO_BYTES bytes)."""
    raw = bytes(info_bytes.cpu().numpy().tobytes())
    n = len(raw) // FIT_INFO_BYTES
    out = []
    for i in range(n):
        rec = vs_fit_info.from_buffer_copy(raw[i * FIT_INFO_BYTES:(i + 1) * FIT_INFO_BYTES])
        out.append({k: getattr(rec, k) for k in FIT_INFO_FIELDS if k != "pad"})
    return out
