// warp_frame: inverse-mapped bilinear warp of 8-bit frames, all items of a batch in one launch.
//
// A 256-thread workgroup covers a 256 x 16 output tile; each thread produces 4 consecutive pixels
// in each of 4 rows, stored as one 32-bit word per row when the row allows it. The 2x3 matrix is
// inverted in binary64 once per thread; per-pixel source coordinates are FP32. The source map is
// affine, so the extreme source coordinates of a thread's 4x4 block are at its corners: when all
// four corners map inside [0, W-2] x [0, H-2], every 2x2 source footprint of the block is inside
// the frame and the thread takes a path without per-pixel border tests, reading through a buffer
// descriptor with 32-bit offsets. Other threads take the general path (border value outside).
// Values are rounded half up: floor(v + 0.5) is an integer in [0, 255], packed exactly.
#include "vs_common.hpp"

namespace {

constexpr int TW = 256, TH = 16;
constexpr uint32_t RSRC_WORD3 = 0x00020000;   // raw (untyped) buffer access on gfx9-family parts

__device__ __forceinline__ float lerp(float u, float v, float t) { return fmaf(t, v - u, u); }

__global__ __launch_bounds__(256) void warp_kernel(const uint8_t* __restrict__ src, int64_t src_stride, int W, int H,
                                                   int src_pitch, const double* __restrict__ mats, int64_t mat_stride,
                                                   uint8_t* __restrict__ dst, int64_t dst_stride, int dst_pitch,
                                                   int border, int tiles_x, int tiles_y)
{
    const int tiles = tiles_x * tiles_y;
    const int item = blockIdx.x / tiles, tile = blockIdx.x - item * tiles;
    const int ty = tile / tiles_x, tx = tile - ty * tiles_x;
    const int x4 = tx * TW + (threadIdx.x & 63) * 4;
    const int ybase = ty * TH + (threadIdx.x >> 6) * 4;
    if (x4 >= W || ybase >= H) return;
    const double* M = mats + item * mat_stride;
    const double rdet = 1.0 / (M[0] * M[4] - M[1] * M[3]);
    const double i00 = M[4] * rdet, i01 = -M[1] * rdet, i10 = -M[3] * rdet, i11 = M[0] * rdet;
    const double i02 = -(i00 * M[2] + i01 * M[5]);
    const double i12 = -(i10 * M[2] + i11 * M[5]);
    const float f00 = (float)i00, f01 = (float)i01, f02 = (float)i02;
    const float f10 = (float)i10, f11 = (float)i11, f12 = (float)i12;
    const uint8_t* s = src + item * src_stride;
    const int nx = W - x4 < 4 ? W - x4 : 4;
    const int ny = H - ybase < 4 ? H - ybase : 4;
    uint8_t* drow = dst + item * dst_stride + (int64_t)ybase * dst_pitch + x4;
    const bool word_store = nx == 4 && (reinterpret_cast<uintptr_t>(drow) & 3) == 0 && (dst_pitch & 3) == 0;

    // corners of the block in source coordinates
    bool inside = true;
#pragma unroll
    for (int cy = 0; cy < 2; ++cy)
#pragma unroll
        for (int cx = 0; cx < 2; ++cx) {
            const float fx = (float)(x4 + 3 * cx), fy = (float)(ybase + 3 * cy);
            const float sx = fmaf(f00, fx, fmaf(f01, fy, f02));
            const float sy = fmaf(f10, fx, fmaf(f11, fy, f12));
            inside = inside && sx >= 0.0f && sy >= 0.0f && sx < (float)(W - 1) && sy < (float)(H - 1);
        }

    if (inside) {
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t*>(s), (short)0,
                                                                            src_pitch * H, RSRC_WORD3);
        for (int r = 0; r < ny; ++r) {
            const float fy = (float)(ybase + r);
            const float bx = fmaf(f01, fy, f02), by = fmaf(f11, fy, f12);
            uint32_t packed = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float fx = (float)(x4 + q);
                const float sx = fmaf(f00, fx, bx);
                const float sy = fmaf(f10, fx, by);
                const float x0 = floorf(sx), y0 = floorf(sy);
                const float a = sx - x0, b = sy - y0;
                const int off = (int)__umul24((unsigned)(int)y0, (unsigned)src_pitch) + (int)x0;
                const float v00 = (float)__builtin_amdgcn_raw_buffer_load_b8(rs, off, 0, 0);
                const float v10 = (float)__builtin_amdgcn_raw_buffer_load_b8(rs, off + 1, 0, 0);
                const float v01 = (float)__builtin_amdgcn_raw_buffer_load_b8(rs, off + src_pitch, 0, 0);
                const float v11 = (float)__builtin_amdgcn_raw_buffer_load_b8(rs, off + src_pitch + 1, 0, 0);
                const float v = lerp(lerp(v00, v10, a), lerp(v01, v11, a), b);
                packed = __builtin_amdgcn_cvt_pk_u8_f32(floorf(v + 0.5f), q, packed);
            }
            uint8_t* out = drow + (int64_t)r * dst_pitch;
            if (word_store) *reinterpret_cast<uint32_t*>(out) = packed;
            else
                for (int q = 0; q < nx; ++q) out[q] = (uint8_t)(packed >> (8 * q));
        }
        return;
    }

    const float bord = (float)border;
    const float fW = (float)W, fH = (float)H;
    for (int r = 0; r < ny; ++r) {
        const int y = ybase + r;
        const float fy = (float)y;
        const float bx = fmaf(f01, fy, f02), by = fmaf(f11, fy, f12);
        uint32_t packed = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float fx = (float)(x4 + q);
            const float sx = fmaf(f00, fx, bx);
            const float sy = fmaf(f10, fx, by);
            uint32_t o = (uint32_t)border;
            if (sx > -1.0f && sx < fW && sy > -1.0f && sy < fH) {
                const float x0 = floorf(sx), y0 = floorf(sy);
                const float a = sx - x0, b = sy - y0;
                const int xi = (int)x0, yi = (int)y0;
                const bool xin0 = xi >= 0, xin1 = xi + 1 < W, yin0 = yi >= 0, yin1 = yi + 1 < H;
                const uint8_t* r0 = s + (int64_t)yi * src_pitch + xi;
                const float v00 = (xin0 && yin0) ? (float)r0[0] : bord;
                const float v10 = (xin1 && yin0) ? (float)r0[1] : bord;
                const float v01 = (xin0 && yin1) ? (float)r0[src_pitch] : bord;
                const float v11 = (xin1 && yin1) ? (float)r0[src_pitch + 1] : bord;
                const float v = lerp(lerp(v00, v10, a), lerp(v01, v11, a), b);
                o = (uint32_t)fminf(fmaxf(floorf(v + 0.5f), 0.0f), 255.0f);
            }
            packed |= o << (8 * q);
        }
        uint8_t* out = drow + (int64_t)r * dst_pitch;
        if (word_store) *reinterpret_cast<uint32_t*>(out) = packed;
        else
            for (int q = 0; q < nx; ++q) out[q] = (uint8_t)(packed >> (8 * q));
    }
}

}  // namespace

extern "C" int vs_warp_frame(const uint8_t* src, int64_t src_stride, int32_t width, int32_t height, int32_t src_pitch,
                             const double* mats, int64_t mat_stride, uint8_t* dst, int64_t dst_stride, int32_t dst_pitch,
                             int32_t n, int32_t border, void* stream)
{
    if (n < 0 || width <= 0 || height <= 0 || src_pitch < width || dst_pitch < width)
        return vs::set_error(VS_ERR_INVALID, "vs_warp_frame: bad size");
    if (n == 0) return VS_OK;
    if (!src || !mats || !dst) return vs::set_error(VS_ERR_INVALID, "vs_warp_frame: null argument");
    if (border < 0 || border > 255) return vs::set_error(VS_ERR_INVALID, "vs_warp_frame: border must be 0..255");
    if (n > 65535) return vs::set_error(VS_ERR_INVALID, "vs_warp_frame: more than 65535 items");
    if ((int64_t)src_pitch * height >= ((int64_t)1 << 31))
        return vs::set_error(VS_ERR_UNSUPPORTED, "vs_warp_frame: frame larger than 2 GiB");
    if (n > 1 && (mat_stride < 6 || src_stride < (int64_t)src_pitch * height || dst_stride < (int64_t)dst_pitch * height))
        return vs::set_error(VS_ERR_INVALID, "vs_warp_frame: strides overlap items");
    const int tiles_x = (width + TW - 1) / TW, tiles_y = (height + TH - 1) / TH;
    const int64_t nblk = (int64_t)n * tiles_x * tiles_y;
    if (nblk > 0x7fffffff) return vs::set_error(VS_ERR_INVALID, "vs_warp_frame: grid too large");
    warp_kernel<<<(unsigned)nblk, 256, 0, vs::as_stream(stream)>>>(src, src_stride, width, height, src_pitch, mats,
                                                                   mat_stride, dst, dst_stride, dst_pitch, border,
                                                                   tiles_x, tiles_y);
    return vs::check_launch("vs_warp_frame");
}
