// build_pyramid: binomial (1 4 6 4 1)^2 / 256 reduce, one level per launch, all items of the batch
// in the same launch.
//
// Each 256-thread workgroup produces a 128 x 32 tile of level l+1. It stages the (2*128+3) x
// (2*32+3) input window of level l in LDS: interior tiles with aligned 32-bit loads (rows of 66
// words), tiles touching the border byte by byte with reflect-101 indices. It then filters rows
// into 16-bit horizontal sums (exact: <= 16 * 255), then columns into 32-bit totals, and rounds
// once. The result is bit-identical to the direct 5x5 integer sum. The tiles of one frame run on
// one XCD when the batch has at least 8 frames, so tile halos are shared in that XCD's L2.
#include "vs_common.hpp"

namespace {

constexpr int TW = 128;                // output tile width
constexpr int TH = 32;                 // output tile height
constexpr int IW = 2 * TW + 3;         // input columns 2*x0-2 .. 2*(x0+TW-1)+2
constexpr int IH = 2 * TH + 3;
constexpr int NWORD = (IW + 3) / 4 + 1;   // 32-bit words covering IW bytes from a 4-aligned start
constexpr int IWP = 4 * NWORD;            // LDS row pitch (bytes)

__device__ __forceinline__ int refl101_clamped(int t, int n)
{
    if (t < 0) t = -t;
    if (t >= n) t = 2 * n - 2 - t;
    return vs::clampi(t, 0, n - 1);    // rows/columns only used by outputs past the edge
}

__global__ __launch_bounds__(256) void pyr_down_kernel(const uint8_t* __restrict__ src, int64_t src_stride,
                                                        int src_pitch, int sw, int sh, uint8_t* __restrict__ dst,
                                                        int64_t dst_stride, int dst_pitch, int dw, int dh, int n_items,
                                                        int tiles_x, int tiles_y, int by_xcd, int word_ok)
{
    __shared__ __attribute__((aligned(16))) uint8_t tin[IH][IWP];
    __shared__ uint16_t hsum[IH][TW];
    int item, tile;
    if (!vs::xcd_map(blockIdx.x, n_items, tiles_x * tiles_y, by_xcd != 0, item, tile)) return;
    const int ty = tile / tiles_x, tx = tile - ty * tiles_x;
    const uint8_t* s = src + item * src_stride;
    uint8_t* d = dst + item * dst_stride;
    const int ox = tx * TW, oy = ty * TH;
    const int ix0 = 2 * ox - 2, iy0 = 2 * oy - 2;
    const int tid = threadIdx.x;
    const int a0 = ix0 & ~3;                 // aligned start of the word path
    int shift = 0;                           // byte offset of input column 0 inside an LDS row
    const bool interior = word_ok && ix0 >= 0 && iy0 >= 0 && a0 + 4 * NWORD <= sw && iy0 + IH <= sh;
    if (interior) {
        shift = ix0 - a0;
        for (int k = tid; k < IH * NWORD; k += 256) {
            const int r = k / NWORD, w = k - r * NWORD;
            const uint32_t v = *reinterpret_cast<const uint32_t*>(s + (int64_t)(iy0 + r) * src_pitch + a0 + 4 * w);
            *reinterpret_cast<uint32_t*>(&tin[r][4 * w]) = v;
        }
    } else {
        for (int k = tid; k < IH * IW; k += 256) {
            const int r = k / IW, c = k - r * IW;
            const int sy = refl101_clamped(iy0 + r, sh);
            const int sx = refl101_clamped(ix0 + c, sw);
            tin[r][c] = s[(int64_t)sy * src_pitch + sx];
        }
    }
    __syncthreads();
    for (int k = tid; k < IH * TW; k += 256) {
        const int r = k / TW, c = k - r * TW;
        const uint8_t* row = &tin[r][2 * c + shift];
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
    const bool by_xcd = n >= VS_XCD_MIN_ITEMS;
    for (int l = 1; l < layout->levels; ++l) {
        const uint8_t* src = (l == 1) ? frames : pyrs + layout->offset[l - 1];
        const int64_t sstride = (l == 1) ? frame_stride : pyr_stride;
        const int spitch = layout->pitch[l - 1];
        const int dw = layout->width[l], dh = layout->height[l];
        const int tiles_x = (dw + TW - 1) / TW, tiles_y = (dh + TH - 1) / TH;
        // 32-bit loads need 4-byte aligned rows in every item
        const bool word_ok = (spitch % 4 == 0) && (reinterpret_cast<uintptr_t>(src) % 4 == 0) &&
                             (n == 1 || sstride % 4 == 0);
        const int64_t nblk = vs::xcd_grid(n, tiles_x * tiles_y, by_xcd);
        pyr_down_kernel<<<(unsigned)nblk, 256, 0, s>>>(src, sstride, spitch, layout->width[l - 1],
                                                       layout->height[l - 1], pyrs + layout->offset[l], pyr_stride,
                                                       layout->pitch[l], dw, dh, n, tiles_x, tiles_y, by_xcd, word_ok);
        int e = vs::check_launch("vs_build_pyramid");
        if (e) return e;
    }
    return VS_OK;
}
