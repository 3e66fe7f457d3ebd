// build_pyramid: binomial (1 4 6 4 1)^2 / 256 reduce, one level per launch, all items of the batch
// in the same launch (grid.z = item).
//
// Each 256-thread workgroup produces a 64 x 32 tile of level l+1. It stages the (2*64+3) x (2*32+3)
// input window of level l in LDS (borders reflected without repeating the edge), filters rows into
// 16-bit horizontal sums (exact: <= 16 * 255), then columns into 32-bit totals, and rounds once.
// The result is bit-identical to the direct 5x5 integer sum.
#include "vs_common.hpp"

namespace {

constexpr int TW = 64;                 // output tile width
constexpr int TH = 32;                 // output tile height
constexpr int IW = 2 * TW + 3;         // input columns 2*x0-2 .. 2*(x0+TW-1)+2
constexpr int IH = 2 * TH + 3;
constexpr int IWP = 132;               // padded LDS row

__device__ __forceinline__ int refl101_clamped(int t, int n)
{
    if (t < 0) t = -t;
    if (t >= n) t = 2 * n - 2 - t;
    return vs::clampi(t, 0, n - 1);    // rows/columns only used by outputs past the edge
}

__global__ __launch_bounds__(256) void pyr_down_kernel(const uint8_t* __restrict__ src, int64_t src_stride,
                                                        int src_pitch, int sw, int sh, uint8_t* __restrict__ dst,
                                                        int64_t dst_stride, int dst_pitch, int dw, int dh)
{
    __shared__ uint8_t tin[IH][IWP];
    __shared__ uint16_t hsum[IH][TW];
    const int item = blockIdx.z;
    const uint8_t* s = src + item * src_stride;
    uint8_t* d = dst + item * dst_stride;
    const int ox = blockIdx.x * TW, oy = blockIdx.y * TH;
    const int ix0 = 2 * ox - 2, iy0 = 2 * oy - 2;
    const int tid = threadIdx.x;

    for (int k = tid; k < IH * IW; k += 256) {
        const int r = k / IW, c = k - r * IW;
        const int sy = refl101_clamped(iy0 + r, sh);
        const int sx = refl101_clamped(ix0 + c, sw);
        tin[r][c] = s[(int64_t)sy * src_pitch + sx];
    }
    __syncthreads();
    for (int k = tid; k < IH * TW; k += 256) {
        const int r = k / TW, c = k - r * TW;
        const uint8_t* row = &tin[r][2 * c];
        hsum[r][c] = (uint16_t)(row[0] + 4 * row[1] + 6 * row[2] + 4 * row[3] + row[4]);
    }
    __syncthreads();
    for (int k = tid; k < TH * TW; k += 256) {
        const int r = k / TW, c = k - r * TW;
        const int x = ox + c, y = oy + r;
        if (x >= dw || y >= dh) continue;
        const uint32_t v = hsum[2 * r][c] + 4u * hsum[2 * r + 1][c] + 6u * hsum[2 * r + 2][c] +
                           4u * hsum[2 * r + 3][c] + hsum[2 * r + 4][c];
        d[(int64_t)y * dst_pitch + x] = (uint8_t)((v + 128u) >> 8);
    }
}

}  // namespace

extern "C" int vs_build_pyramid(const uint8_t* frames, int64_t frame_stride, uint8_t* pyrs, int64_t pyr_stride,
                                int32_t n, const vs_pyramid* layout, void* stream)
{
    if (!layout || (n > 0 && (!frames || !pyrs)))
        return vs::set_error(VS_ERR_INVALID, "vs_build_pyramid: null argument");
    if (n < 0 || layout->levels < 1 || layout->levels > VS_MAX_LEVELS)
        return vs::set_error(VS_ERR_INVALID, "vs_build_pyramid: bad count or levels");
    if (n == 0 || layout->levels == 1) return VS_OK;
    if (n > 65535) return vs::set_error(VS_ERR_INVALID, "vs_build_pyramid: more than 65535 items");
    if (n > 1 && (frame_stride < (int64_t)layout->pitch[0] * layout->height[0] || pyr_stride < layout->bytes))
        return vs::set_error(VS_ERR_INVALID, "vs_build_pyramid: strides overlap items");
    hipStream_t s = vs::as_stream(stream);
    for (int l = 1; l < layout->levels; ++l) {
        const uint8_t* src = (l == 1) ? frames : pyrs + layout->offset[l - 1];
        const int64_t sstride = (l == 1) ? frame_stride : pyr_stride;
        const int dw = layout->width[l], dh = layout->height[l];
        dim3 grid((dw + TW - 1) / TW, (dh + TH - 1) / TH, n);
        pyr_down_kernel<<<grid, 256, 0, s>>>(src, sstride, layout->pitch[l - 1], layout->width[l - 1],
                                             layout->height[l - 1], pyrs + layout->offset[l], pyr_stride,
                                             layout->pitch[l], dw, dh);
        int e = vs::check_launch("vs_build_pyramid");
        if (e) return e;
    }
    return VS_OK;
}
