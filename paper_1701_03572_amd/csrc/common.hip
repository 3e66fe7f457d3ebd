// Error reporting, version, launch tuning and the pyramid layout query of libvstab.
#include <atomic>
#include <cstdarg>

#include "vs_common.hpp"

namespace vs {

static thread_local char g_err[512] = "";

int set_error(int code, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

int check_launch(const char* what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(VS_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
    return VS_OK;
}

// launch tuning: speed-only choices, read by each call when it launches
static std::atomic<int> g_xcd_pyr{VS_XCD_MIN_ITEMS}, g_xcd_lk{VS_XCD_MIN_ITEMS}, g_xcd_warp{VS_XCD_MIN_ITEMS};
static std::atomic<int> g_lk_ppg{1};
static std::atomic<int> g_det_rows{0}, g_fit_groups{2048};

int xcd_min_items(int kernel)
{
    switch (kernel) {
    case XCD_PYRAMID: return g_xcd_pyr.load(std::memory_order_relaxed);
    case XCD_LK: return g_xcd_lk.load(std::memory_order_relaxed);
    default: return g_xcd_warp.load(std::memory_order_relaxed);
    }
}

int lk_points_per_group() { return g_lk_ppg.load(std::memory_order_relaxed); }

int detect_segment_rows(int n_items, int few_rows, int many_rows)
{
    const int r = g_det_rows.load(std::memory_order_relaxed);
    return r ? r : (n_items <= 8 ? few_rows : many_rows);
}

int fit_groups_in_flight() { return g_fit_groups.load(std::memory_order_relaxed); }

}  // namespace vs

extern "C" int vs_set_tuning(const vs_tuning* t)
{
    vs_tuning v{0, 0, 0, 0, 0, 0};
    if (t) v = *t;
    const int xs[3] = {v.xcd_min_items_pyramid, v.xcd_min_items_lk, v.xcd_min_items_warp};
    for (int x : xs)
        if (x < 0 || x > 65536) return vs::set_error(VS_ERR_INVALID, "vs_set_tuning: xcd_min_items must be 0..65536");
    if (!(v.lk_points_per_group == 0 || v.lk_points_per_group == 1 || v.lk_points_per_group == 2 ||
          v.lk_points_per_group == 4))
        return vs::set_error(VS_ERR_INVALID, "vs_set_tuning: lk_points_per_group must be 0, 1, 2 or 4");
    if (!(v.detect_segment_rows == 0 || (v.detect_segment_rows >= 12 && v.detect_segment_rows <= 240)))
        return vs::set_error(VS_ERR_INVALID, "vs_set_tuning: detect_segment_rows must be 0 or 12..240");
    if (!(v.fit_groups_in_flight == 0 || (v.fit_groups_in_flight >= 64 && v.fit_groups_in_flight <= 16384)))
        return vs::set_error(VS_ERR_INVALID, "vs_set_tuning: fit_groups_in_flight must be 0 or 64..16384");
    vs::g_xcd_pyr.store(xs[0] ? xs[0] : VS_XCD_MIN_ITEMS);
    vs::g_xcd_lk.store(xs[1] ? xs[1] : VS_XCD_MIN_ITEMS);
    vs::g_xcd_warp.store(xs[2] ? xs[2] : VS_XCD_MIN_ITEMS);
    vs::g_lk_ppg.store(v.lk_points_per_group ? v.lk_points_per_group : 1);
    vs::g_det_rows.store(v.detect_segment_rows);
    vs::g_fit_groups.store(v.fit_groups_in_flight ? v.fit_groups_in_flight : 2048);
    return VS_OK;
}

extern "C" int vs_get_tuning(vs_tuning* t)
{
    if (!t) return vs::set_error(VS_ERR_INVALID, "vs_get_tuning: null output");
    t->xcd_min_items_pyramid = vs::g_xcd_pyr.load();
    t->xcd_min_items_lk = vs::g_xcd_lk.load();
    t->xcd_min_items_warp = vs::g_xcd_warp.load();
    t->lk_points_per_group = vs::g_lk_ppg.load();
    t->detect_segment_rows = vs::g_det_rows.load();
    t->fit_groups_in_flight = vs::g_fit_groups.load();
    return VS_OK;
}

extern "C" const char* vs_last_error(void) { return vs::g_err; }

extern "C" int vs_version(void) { return 1; }

// Level sizes halve with rounding up; each level above 0 gets a pitch rounded to 64 bytes and a
// 256-byte aligned offset in one buffer.
extern "C" int vs_pyramid_layout(int32_t width, int32_t height, int32_t pitch0, int32_t levels, vs_pyramid* out)
{
    if (!out) return vs::set_error(VS_ERR_INVALID, "vs_pyramid_layout: null output");
    if (levels < 1) return vs::set_error(VS_ERR_INVALID, "vs_pyramid_layout: levels < 1");
    if (levels > VS_MAX_LEVELS) return vs::set_error(VS_ERR_UNSUPPORTED, "vs_pyramid_layout: levels > %d", VS_MAX_LEVELS);
    if (pitch0 < width) return vs::set_error(VS_ERR_INVALID, "vs_pyramid_layout: pitch < width");
    std::memset(out, 0, sizeof(*out));
    out->levels = levels;
    int w = width, h = height;
    int64_t off = 0;
    for (int l = 0; l < levels; ++l) {
        if (w < 16 || h < 16)
            return vs::set_error(VS_ERR_INVALID, "vs_pyramid_layout: level %d is %dx%d (< 16)", l, w, h);
        out->width[l] = w;
        out->height[l] = h;
        if (l == 0) {
            out->pitch[0] = pitch0;
            out->offset[0] = 0;
        } else {
            const int p = (w + 63) & ~63;
            out->pitch[l] = p;
            out->offset[l] = off;
            off += ((int64_t)p * h + 255) & ~(int64_t)255;
        }
        w = (w + 1) / 2;
        h = (h + 1) / 2;
    }
    out->bytes = off;
    return VS_OK;
}
