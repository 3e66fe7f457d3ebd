// batch_push: the per-frame path of the real-time version (Section 6) for many streams at once. One
// call processes the next frame of every listed stream of a batch with one launch per stage: the
// pyramids, the tracking of the previous frames' points with the backward check (Sections 3.2, 4.1),
// the fits with the dwell switch and the skip rule (Section 4), the smoother's step (Sections 5.1, 6),
// the warps of the emitted frames (Section 5) and the re-detections (every redetect_every frames, and
// after a pair with too few valid points).
//
// Each attached stream has a device descriptor (its vs_stream buffers, its corner budget, RANSAC
// seed and stream id, and its device-side frame counter); a step's items are descriptor slots
// written by the step's first kernel. The kernels are the single-stream ones, addressed per item
// through the descriptors, so every stream's results are those of vs_stream_push on the same
// frames, bit for bit. The launches of a step depend only on the slots, so a step over a fixed set of
// streams can be captured once and replayed frame after frame.
#include <cstddef>

#include "vs_common.hpp"

namespace {

constexpr int SETUP_CHUNK = 64;

struct SlotChunk {
    int32_t slot[SETUP_CHUNK];
};

// writes the step's slots [first, first + n) and clears the valid-point counters of the items that
// track a pair in this step (j > 0); the tracker adds to them
__global__ void step_setup_kernel(SlotChunk c, int first, int n, int32_t* slot_buf, vs::StepStream* desc)
{
    const int k = threadIdx.x;
    if (k >= n) return;
    const int32_t sl = c.slot[k];
    slot_buf[first + k] = sl;
    vs::StepStream& d = desc[sl];
    if (d.next_frame > 0) *d.n_valid = 0;
}

__global__ void step_advance_kernel(vs::StepView v, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v.s(i).next_frame += 1;
}

__global__ void desc_write_kernel(vs::StepStream d, vs::StepStream* dst) { *dst = d; }

int lag_of(const vs_stream* s) { return s->smooth.mode == VS_SMOOTH_CENTERED ? s->smooth.radius : 0; }

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
    size_t desc, slots, fit, det, total;
};

Layout ws_layout(const vs_stream* p, int max_streams, int detect_chunk)
{
    Layout L;
    L.desc = 0;
    L.slots = align256(sizeof(vs::StepStream) * (size_t)max_streams);
    L.fit = L.slots + align256(sizeof(int32_t) * (size_t)max_streams);
    L.det = L.fit + align256(vs::step_fit_workspace(max_streams, p->capacity));
    L.total = L.det + vs_detect_workspace(p->width, p->height, detect_chunk);
    return L;
}

bool same_layout(const vs_pyramid& a, const vs_pyramid& b)
{
    if (a.levels != b.levels || a.bytes != b.bytes) return false;
    for (int l = 0; l < a.levels; ++l)
        if (a.width[l] != b.width[l] || a.height[l] != b.height[l] || a.pitch[l] != b.pitch[l] ||
            a.offset[l] != b.offset[l])
            return false;
    return true;
}

// everything but the per-stream budget, seed and stream id must equal the batch's prototype
bool same_class(const vs_stream* a, const vs_stream* b)
{
    const vs_detect_params &da = a->detect, &db = b->detect;
    const vs_lk_params &la = a->lk, &lb = b->lk;
    const vs_fit_params &fa = a->fit, &fb = b->fit;
    const vs_smooth_params &sa = a->smooth, &sb = b->smooth;
    return a->width == b->width && a->height == b->height && same_layout(a->layout, b->layout) &&
           a->capacity == b->capacity && a->redetect_every == b->redetect_every && a->min_valid == b->min_valid &&
           a->border == b->border && a->photo_steps == b->photo_steps && da.quality == db.quality &&
           da.min_dist == db.min_dist && da.roi_mx == db.roi_mx && da.roi_my == db.roi_my &&
           da.max_corners_per_item == nullptr && db.max_corners_per_item == nullptr && la.win_half == lb.win_half &&
           la.max_iter == lb.max_iter && la.eps == lb.eps && la.min_eig == lb.min_eig && la.fb == lb.fb &&
           la.fb_thresh == lb.fb_thresh && fa.model == fb.model && fa.ransac_iters == fb.ransac_iters &&
           fa.inlier_thresh == fb.inlier_thresh && fa.min_valid == fb.min_valid && fa.dwell == fb.dwell &&
           fa.cx == fb.cx && fa.cy == fb.cy && sa.mode == sb.mode && sa.radius == sb.radius &&
           sa.kalman_ratio == sb.kalman_ratio && sa.crop == sb.crop && sa.cx == sb.cx && sa.cy == sb.cy;
}

vs::StepView view_of(const vs_batch* b)
{
    const Layout L = ws_layout(&b->proto, b->max_streams, b->detect_chunk);
    uint8_t* w8 = static_cast<uint8_t*>(b->workspace);
    vs::StepView v;
    v.desc = reinterpret_cast<vs::StepStream*>(w8 + L.desc);
    v.slot = reinterpret_cast<const int32_t*>(w8 + L.slots);
    v.plane = (int64_t)b->proto.width * b->proto.height;
    v.pyr_bytes = b->proto.layout.bytes;
    v.capacity = b->proto.capacity;
    v.lag = lag_of(&b->proto);
    v.redetect_every = b->proto.redetect_every;
    v.min_valid = b->proto.min_valid;
    return v;
}

// the host-side progress of one pushed frame, as vs_stream_push keeps it
void note_push(vs_stream* s, int64_t plane, int64_t* first, int32_t* count)
{
    const int lag = lag_of(s);
    const int64_t j = s->next_frame;
    s->frames[j % (lag + 2)] = s->ring + (j % s->ring_len) * plane;
    s->next_frame = j + 1;
    int64_t end = lag ? s->next_frame - lag : s->next_frame;
    if (end < s->emitted) end = s->emitted;
    *first = s->emitted;
    *count = (int32_t)(end - s->emitted);
    s->emitted = end;
}

int check_items(const vs_batch* b, int32_t n, const int32_t* slots, const char* who)
{
    if (!b || !b->workspace) return vs::set_error(VS_ERR_INVALID, "%s: batch not initialised", who);
    if (n < 0 || n > b->max_streams) return vs::set_error(VS_ERR_INVALID, "%s: bad item count %d", who, n);
    if (n > 0 && !slots) return vs::set_error(VS_ERR_INVALID, "%s: null slots", who);
    bool seen[VS_BATCH_MAX_STREAMS] = {};
    for (int k = 0; k < n; ++k) {
        const int32_t sl = slots[k];
        if (sl < 0 || sl >= b->max_streams || !b->attached[sl])
            return vs::set_error(VS_ERR_INVALID, "%s: slot %d is not attached", who, sl);
        if (seen[sl]) return vs::set_error(VS_ERR_INVALID, "%s: slot %d listed twice", who, sl);
        seen[sl] = true;
    }
    return VS_OK;
}

}  // namespace

extern "C" size_t vs_batch_workspace(const vs_stream* proto, int32_t max_streams, int32_t detect_chunk)
{
    if (!proto || max_streams <= 0 || max_streams > VS_BATCH_MAX_STREAMS || detect_chunk <= 0 ||
        proto->width <= 0 || proto->height <= 0 || proto->capacity <= 0)
        return 0;
    return ws_layout(proto, max_streams, detect_chunk).total;
}

extern "C" int vs_batch_init(vs_batch* b, const vs_stream* proto, int32_t max_streams, int32_t detect_chunk,
                             void* workspace, size_t ws_bytes)
{
    if (!b || !proto) return vs::set_error(VS_ERR_INVALID, "vs_batch_init: null argument");
    if (max_streams <= 0 || max_streams > VS_BATCH_MAX_STREAMS || detect_chunk <= 0 || detect_chunk > max_streams)
        return vs::set_error(VS_ERR_INVALID, "vs_batch_init: need 0 < detect_chunk <= max_streams <= %d",
                             VS_BATCH_MAX_STREAMS);
    if (proto->photo_steps != 0)
        return vs::set_error(VS_ERR_UNSUPPORTED, "vs_batch_init: the batched step has no photometric refinement");
    if (proto->width <= 0 || proto->height <= 0 || proto->capacity <= 0 || proto->capacity > VS_MAX_CORNERS ||
        proto->redetect_every <= 0 || proto->layout.width[0] != proto->width || proto->layout.height[0] != proto->height ||
        proto->layout.pitch[0] != proto->width)
        return vs::set_error(VS_ERR_INVALID, "vs_batch_init: bad geometry, capacity or cadence");
    if (proto->smooth.radius < 0 || proto->smooth.radius > 127 || lag_of(proto) + 2 > VS_STREAM_MAX_FRAMES)
        return vs::set_error(VS_ERR_INVALID, "vs_batch_init: smoothing radius must be 0..127");
    const size_t need = vs_batch_workspace(proto, max_streams, detect_chunk);
    if (!workspace || ws_bytes < need)
        return vs::set_error(VS_ERR_WORKSPACE, "vs_batch_init: workspace %zu < %zu", ws_bytes, need);
    if (reinterpret_cast<uintptr_t>(workspace) & 255)
        return vs::set_error(VS_ERR_INVALID, "vs_batch_init: workspace must be 256-byte aligned");
    b->proto = *proto;
    b->max_streams = max_streams;
    b->detect_chunk = detect_chunk;
    b->workspace = workspace;
    b->ws_bytes = ws_bytes;
    b->ready_event = nullptr;
    for (int i = 0; i < VS_BATCH_MAX_STREAMS; ++i) b->attached[i] = nullptr;
    return VS_OK;
}

extern "C" int vs_batch_attach(vs_batch* b, int32_t slot, vs_stream* s, void* stream)
{
    if (!b || !b->workspace || !s) return vs::set_error(VS_ERR_INVALID, "vs_batch_attach: null argument");
    if (slot < 0 || slot >= b->max_streams || b->attached[slot])
        return vs::set_error(VS_ERR_INVALID, "vs_batch_attach: slot %d is out of range or taken", slot);
    if (!same_class(s, &b->proto))
        return vs::set_error(VS_ERR_INVALID, "vs_batch_attach: the stream's geometry or shared parameters differ from "
                                             "the batch's");
    if (s->detect.max_corners < 0 || s->detect.max_corners > s->capacity)
        return vs::set_error(VS_ERR_INVALID, "vs_batch_attach: need 0 <= max_corners <= capacity");
    const int lag = lag_of(s);
    if (!s->ring || s->ring_len < lag + 2 || (reinterpret_cast<uintptr_t>(s->ring) & 15))
        return vs::set_error(VS_ERR_INVALID, "vs_batch_attach: the stream needs a 16-byte aligned frame ring of at "
                                             "least %d frames", lag + 2);
    if (!s->pyr || (reinterpret_cast<uintptr_t>(s->pyr) & 255) || (s->layout.bytes & 255))
        return vs::set_error(VS_ERR_INVALID, "vs_batch_attach: the pyramids must be 256-byte aligned");
    for (int i = 0; i < b->max_streams; ++i)
        if (b->attached[i] == s) return vs::set_error(VS_ERR_INVALID, "vs_batch_attach: stream already attached");
    int rc = vs_stream_reset(s, stream);   // validates the stream's buffers, starts it at frame 0
    if (rc) return rc;
    vs::StepStream d{};
    d.ring = s->ring;
    d.pyr = s->pyr;
    d.pts = s->pts;
    d.alive = s->alive;
    d.dst = s->dst;
    d.status = s->status;
    d.fb_err = s->fb_err;
    d.n_valid = s->n_valid;
    d.count = s->count;
    d.fit_state = s->fit_state;
    d.pair_params = s->pair_params;
    d.affine6 = s->affine6;
    d.info = s->info;
    d.inliers = s->inliers;
    d.traj_state = s->traj_state;
    d.mats = s->mats;
    d.n_emitted = s->n_emitted;
    d.first_frame = s->first_frame;
    d.out = s->out;
    d.next_frame = 0;
    d.ring_len = s->ring_len;
    d.out_slots = s->out_slots;
    d.max_corners = s->detect.max_corners;
    d.seed = s->fit.seed;
    d.stream_id = s->fit.stream_id;
    if (!d.fb_err || !d.affine6 || !d.inliers)
        return vs::set_error(VS_ERR_INVALID, "vs_batch_attach: the batched step needs fb_err, affine6 and inliers");
    const vs::StepView v = view_of(b);
    desc_write_kernel<<<1, 1, 0, vs::as_stream(stream)>>>(d, v.desc + slot);
    rc = vs::check_launch("vs_batch_attach");
    if (rc) return rc;
    b->attached[slot] = s;
    return VS_OK;
}

extern "C" int vs_batch_detach(vs_batch* b, int32_t slot)
{
    if (!b || slot < 0 || slot >= b->max_streams || !b->attached[slot])
        return vs::set_error(VS_ERR_INVALID, "vs_batch_detach: slot %d is not attached", slot);
    b->attached[slot] = nullptr;
    return VS_OK;
}

extern "C" int vs_batch_push(vs_batch* b, int32_t n, const int32_t* slots, int64_t* first_emitted, int32_t* n_emitted,
                             void* stream)
{
    const char* who = "vs_batch_push";
    int rc = check_items(b, n, slots, who);
    if (rc) return rc;
    if (n == 0) return VS_OK;
    if (!first_emitted || !n_emitted) return vs::set_error(VS_ERR_INVALID, "%s: null output", who);
    hipStream_t st = vs::as_stream(stream);
    const vs_stream& P = b->proto;
    const Layout L = ws_layout(&P, b->max_streams, b->detect_chunk);
    uint8_t* w8 = static_cast<uint8_t*>(b->workspace);
    vs::StepView v = view_of(b);
    int32_t* slot_buf = reinterpret_cast<int32_t*>(w8 + L.slots);
    for (int first = 0; first < n; first += SETUP_CHUNK) {
        const int m = n - first < SETUP_CHUNK ? n - first : SETUP_CHUNK;
        SlotChunk c{};
        for (int k = 0; k < m; ++k) c.slot[k] = slots[first + k];
        step_setup_kernel<<<1, SETUP_CHUNK, 0, st>>>(c, first, m, slot_buf, v.desc);
        if ((rc = vs::check_launch("vs_batch_push(setup)"))) return rc;
    }
    // 16-byte staging loads of frame rows: every frame sits at ring + k * plane with a 16-byte aligned ring
    const bool vec_ok = (P.width % 16) == 0;
    if ((rc = vs::step_pyramid(v, n, P.layout, vec_ok, st))) return rc;
    if ((rc = vs::step_track(v, n, P.layout, P.lk, st))) return rc;
    if ((rc = vs::step_fit(v, n, P.fit, w8 + L.fit, st))) return rc;
    if ((rc = vs::step_smooth(v, n, P.smooth, st))) return rc;
    if ((rc = vs::step_warp(v, n, P.width, P.height, P.border, vec_ok, st))) return rc;
    if (b->ready_event && hipEventRecord(static_cast<hipEvent_t>(b->ready_event), st) != hipSuccess)
        return vs::set_error(VS_ERR_HIP, "%s: hipEventRecord failed", who);
    // the corners detected on frame j serve only the pair (j, j + 1): last, after the ready event
    for (int first = 0; first < n; first += b->detect_chunk) {
        vs::StepView c = v;
        c.slot = v.slot + first;
        const int m = n - first < b->detect_chunk ? n - first : b->detect_chunk;
        if ((rc = vs::step_detect(c, m, P.width, P.height, P.detect, w8 + L.det, st))) return rc;
    }
    step_advance_kernel<<<(n + 63) / 64, 64, 0, st>>>(v, n);
    if ((rc = vs::check_launch("vs_batch_push(advance)"))) return rc;
    const int64_t plane = (int64_t)P.width * P.height;
    for (int k = 0; k < n; ++k) note_push(b->attached[slots[k]], plane, &first_emitted[k], &n_emitted[k]);
    return VS_OK;
}

extern "C" int vs_batch_note_replayed(vs_batch* b, int32_t n, const int32_t* slots, int32_t steps)
{
    int rc = check_items(b, n, slots, "vs_batch_note_replayed");
    if (rc) return rc;
    if (steps < 0) return vs::set_error(VS_ERR_INVALID, "vs_batch_note_replayed: negative step count");
    const int64_t plane = (int64_t)b->proto.width * b->proto.height;
    for (int t = 0; t < steps; ++t)
        for (int k = 0; k < n; ++k) {
            int64_t f;
            int32_t c;
            note_push(b->attached[slots[k]], plane, &f, &c);
        }
    return VS_OK;
}
