// stream_push: the per-frame (real-time) path driven from native code. Each call enqueues every
// launch of one frame through the library's own entry points, with the frame's indices and ring
// positions computed on the host, so a frame costs one call into the library instead of one per
// stage. The sequence of operations is the streaming pipeline's:
//   pyramid(j); j = 0: smoother start; j > 0: track(j - 1 -> j) with the backward check and
//   chaining, fit(pair j - 1), optional photometric refinement, smoother step; then the warps of
//   the frames the smoother emits, the caller's ready event, and last detect(j) (every
//   redetect_every frames and for j = 0, else gated on the device by the pair's valid count):
//   its corners serve only the pair (j, j + 1), so the frame's outputs need not wait for it.
#include <cstddef>

#include "vs_common.hpp"

namespace {

int lag_of(const vs_stream* s) { return s->smooth.mode == VS_SMOOTH_CENTERED ? s->smooth.radius : 0; }

int check(const vs_stream* s)
{
    if (!s) return vs::set_error(VS_ERR_INVALID, "vs_stream: null stream struct");
    if (s->width <= 0 || s->height <= 0 || s->capacity <= 0 || s->out_slots <= 0 || s->redetect_every <= 0)
        return vs::set_error(VS_ERR_INVALID, "vs_stream: bad size, capacity, output slots or cadence");
    if (s->smooth.radius < 0 || s->smooth.radius > 127)
        return vs::set_error(VS_ERR_INVALID, "vs_stream: smoothing radius must be 0..127");
    if (lag_of(s) + 2 > VS_STREAM_MAX_FRAMES) return vs::set_error(VS_ERR_INVALID, "vs_stream: lag too long");
    if (!s->pyr || !s->pts || !s->alive || !s->dst || !s->status || !s->n_valid || !s->count || !s->fit_state ||
        !s->pair_params || !s->info || !s->traj_state || !s->mats || !s->n_emitted || !s->first_frame || !s->out)
        return vs::set_error(VS_ERR_INVALID, "vs_stream: null buffer");
    if (s->photo_steps > 0 && (!s->photo_ws || !s->photo_loss || !s->photo_accepted))
        return vs::set_error(VS_ERR_INVALID, "vs_stream: null photometric buffer");
    return VS_OK;
}

int detect(vs_stream* s, const uint8_t* frame, int slot, bool gated, hipStream_t st)
{
    return vs_detect_corners(frame, 0, s->width, s->height, s->width, 1, 1, gated ? s->n_valid : nullptr, s->min_valid,
                             &s->detect, s->capacity, s->pts + (size_t)slot * s->capacity * 2, nullptr, s->count,
                             s->alive + (size_t)slot * s->capacity, s->detect_ws, s->detect_ws_bytes, st);
}

// warps the frames [emitted, end) with the matrices the smoother's last call wrote to mats[0..]
int emit(vs_stream* s, int64_t end, int64_t* first, int32_t* count, hipStream_t st)
{
    const int ring = lag_of(s) + 2;
    const int64_t plane = (int64_t)s->width * s->height;
    *first = s->emitted;
    *count = (int32_t)(end - s->emitted);
    for (int64_t e = s->emitted, k = 0; e < end; ++e, ++k) {
        const int rc = vs_warp_frame(s->frames[e % ring], 0, s->width, s->height, s->width, s->mats + 6 * k, 6,
                                     s->out + (e % s->out_slots) * plane, 0, s->width, 1, s->border, st);
        if (rc) return rc;
    }
    s->emitted = end;
    return VS_OK;
}

}  // namespace

extern "C" int vs_stream_reset(vs_stream* s, void* stream)
{
    const int e = check(s);
    if (e) return e;
    s->next_frame = 0;
    s->emitted = 0;
    for (int i = 0; i < VS_STREAM_MAX_FRAMES; ++i) s->frames[i] = nullptr;
    const int rc = vs_fit_state_init(s->fit_state, stream);
    return rc ? rc : vs_traj_state_init(s->traj_state, stream);
}

extern "C" int vs_stream_push(vs_stream* s, const uint8_t* frame, int64_t* first_emitted, int32_t* n_emitted,
                              void* stream)
{
    int rc = check(s);
    if (rc) return rc;
    if (!frame || !first_emitted || !n_emitted) return vs::set_error(VS_ERR_INVALID, "vs_stream_push: null argument");
    hipStream_t st = vs::as_stream(stream);
    const int64_t j = s->next_frame;
    const int ring = lag_of(s) + 2;
    const int cur = (int)(j & 1), prev = (int)((j + 1) & 1);
    const int64_t pb = s->layout.bytes;
    uint8_t* pyr_cur = s->pyr + cur * pb;
    if ((rc = vs_build_pyramid(frame, 0, pyr_cur, 0, 1, &s->layout, st))) return rc;
    s->frames[j % ring] = frame;
    if (j == 0) {
        if ((rc = vs_smooth_trajectory(nullptr, 0, 0, &s->smooth, s->traj_state, s->mats, ring, s->n_emitted,
                                       s->first_frame, st)))
            return rc;
    } else {
        const uint8_t* pf = s->frames[(j - 1) % ring];
        const size_t pts2 = (size_t)s->capacity * 2;
        if ((rc = vs_track_lk(pf, s->pyr + prev * pb, frame, pyr_cur, 0, 0, 1, 1, &s->layout, s->pts + prev * pts2,
                              s->alive + (size_t)prev * s->capacity, s->capacity, &s->lk, s->dst, s->status, s->fb_err,
                              s->n_valid, s->pts + cur * pts2, s->alive + (size_t)cur * s->capacity, nullptr, st)))
            return rc;
        if ((rc = vs_fit_motion(s->pts + prev * pts2, s->dst, s->status, s->capacity, 1, &s->fit, j - 1, s->fit_state,
                                s->pair_params, s->affine6, s->info, s->inliers, s->fit_ws, s->fit_ws_bytes, st)))
            return rc;
        if (s->photo_steps > 0) {
            const int32_t* skip = reinterpret_cast<const int32_t*>(reinterpret_cast<const char*>(s->info) +
                                                                   offsetof(vs_fit_info, skipped));
            if ((rc = vs_photometric_refine(pf, frame, 0, s->width, s->height, s->width, 1, s->pair_params,
                                            s->pair_params, 4, VS_PHOTO_FIT, skip, sizeof(vs_fit_info) / 4,
                                            (s->width - 1) / 2.0, (s->height - 1) / 2.0,
                                            (s->width > s->height ? s->width : s->height) / 2.0, &s->photo_omega,
                                            s->photo_steps, s->photo_loss, s->photo_accepted, s->photo_ws,
                                            s->photo_ws_bytes, st)))
                return rc;
        }
        if ((rc = vs_smooth_trajectory(s->pair_params, 1, 0, &s->smooth, s->traj_state, s->mats, ring, s->n_emitted,
                                       s->first_frame, st)))
            return rc;
    }
    s->next_frame = j + 1;
    const int lag = lag_of(s);
    int64_t end = lag ? s->next_frame - lag : s->next_frame;
    if (end < s->emitted) end = s->emitted;
    if ((rc = emit(s, end, first_emitted, n_emitted, st))) return rc;
    if (s->ready_event && hipEventRecord(static_cast<hipEvent_t>(s->ready_event), st) != hipSuccess)
        return vs::set_error(VS_ERR_HIP, "vs_stream_push: hipEventRecord failed");
    return detect(s, frame, cur, j != 0 && j % s->redetect_every != 0, st);
}

extern "C" int vs_stream_flush(vs_stream* s, int64_t* first_emitted, int32_t* n_emitted, void* stream)
{
    int rc = check(s);
    if (rc) return rc;
    if (!first_emitted || !n_emitted) return vs::set_error(VS_ERR_INVALID, "vs_stream_flush: null argument");
    hipStream_t st = vs::as_stream(stream);
    if ((rc = vs_smooth_trajectory(nullptr, 0, 1, &s->smooth, s->traj_state, s->mats, lag_of(s) + 2, s->n_emitted,
                                   s->first_frame, st)))
        return rc;
    return emit(s, s->next_frame, first_emitted, n_emitted, st);
}
