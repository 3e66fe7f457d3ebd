// Error reporting, version and the pyramid layout query of libvstab.
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

}  // namespace vs

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
