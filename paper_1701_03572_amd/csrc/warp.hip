// warp_frame: inverse-mapped bilinear warp of 8-bit frames, all items of a batch in one launch.
//
// A 256-thread workgroup covers 256 x 4 output pixels; each thread produces 4 consecutive pixels
// of one row and stores them as one 32-bit word when the row allows it. The 2x3 matrix is
// inverted in binary64 per thread (a handful of operations), per-pixel coordinates are FP32.
#include "vs_common.hpp"

namespace {

__global__ __launch_bounds__(256) void warp_kernel(const uint8_t* __restrict__ src, int64_t src_stride, int W, int H,
                                                   int src_pitch, const double* __restrict__ mats, int64_t mat_stride,
                                                   uint8_t* __restrict__ dst, int64_t dst_stride, int dst_pitch,
                                                   int border)
{
    const int item = blockIdx.z;
    const int x4 = (blockIdx.x * 64 + (threadIdx.x & 63)) * 4;
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (y >= H || x4 >= W) return;
    const double* M = mats + item * mat_stride;
    const double det = M[0] * M[4] - M[1] * M[3];
    const double i00 = M[4] / det, i01 = -M[1] / det, i10 = -M[3] / det, i11 = M[0] / det;
    const double i02 = -(i00 * M[2] + i01 * M[5]);
    const double i12 = -(i10 * M[2] + i11 * M[5]);
    const float f00 = (float)i00, f01 = (float)i01, f02 = (float)i02;
    const float f10 = (float)i10, f11 = (float)i11, f12 = (float)i12;
    const uint8_t* s = src + item * src_stride;
    uint8_t* d = dst + item * dst_stride + (int64_t)y * dst_pitch;
    const float fy = (float)y;
    const float bx = fmaf(f01, fy, f02), by = fmaf(f11, fy, f12);
    const float bord = (float)border;
    uint32_t packed = 0;
    const int nx = W - x4 < 4 ? W - x4 : 4;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (q >= nx) break;
        const float fx = (float)(x4 + q);
        const float sx = fmaf(f00, fx, bx);
        const float sy = fmaf(f10, fx, by);
        uint32_t o = (uint32_t)border;
        if (sx > -1.0f && sx < (float)W && sy > -1.0f && sy < (float)H) {
            const float x0 = floorf(sx), y0 = floorf(sy);
            const float a = sx - x0, b = sy - y0;
            const int xi = (int)x0, yi = (int)y0;
            const bool xin0 = xi >= 0, xin1 = xi + 1 < W, yin0 = yi >= 0, yin1 = yi + 1 < H;
            const uint8_t* r0 = s + (int64_t)yi * src_pitch;
            const uint8_t* r1 = r0 + src_pitch;
            const float v00 = (xin0 && yin0) ? (float)r0[xi] : bord;
            const float v10 = (xin1 && yin0) ? (float)r0[xi + 1] : bord;
            const float v01 = (xin0 && yin1) ? (float)r1[xi] : bord;
            const float v11 = (xin1 && yin1) ? (float)r1[xi + 1] : bord;
            const float v = (1.0f - b) * ((1.0f - a) * v00 + a * v10) + b * ((1.0f - a) * v01 + a * v11);
            const float r = fminf(fmaxf(floorf(v + 0.5f), 0.0f), 255.0f);
            o = (uint32_t)r;
        }
        packed |= o << (8 * q);
    }
    uint8_t* out = d + x4;
    if (nx == 4 && (reinterpret_cast<uintptr_t>(out) & 3) == 0) {
        *reinterpret_cast<uint32_t*>(out) = packed;
    } else {
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
    if (n > 1 && (mat_stride < 6 || src_stride < (int64_t)src_pitch * height || dst_stride < (int64_t)dst_pitch * height))
        return vs::set_error(VS_ERR_INVALID, "vs_warp_frame: strides overlap items");
    dim3 grid((width + 255) / 256, (height + 3) / 4, n);
    warp_kernel<<<grid, 256, 0, vs::as_stream(stream)>>>(src, src_stride, width, height, src_pitch, mats, mat_stride,
                                                         dst, dst_stride, dst_pitch, border);
    return vs::check_launch("vs_warp_frame");
}
