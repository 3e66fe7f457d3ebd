// build_pyramid: binomial (1 4 6 4 1)^2 / 256 reduce, one level per launch, all items of the batch
// in the same launch.
//
// Each 256-thread workgroup produces a 128 x 32 tile of level l+1 from the (2*128+3) x (2*32+3) input
// window of level l, staged in LDS with 16-byte loads from reflect-101 rows. Columns outside the frame
// are never loaded: a chunk crossing an edge loads its in-frame bytes one by one, and after staging
// the (at most two) reflect-101 columns on each side are copied inside LDS from the columns they
// mirror. Each thread then produces a 4 x 4 block: for each of its 11 input rows
// it forms the 4 horizontal 5-tap sums with byte dot products on aligned LDS words, and it filters
// those sums vertically in registers. All sums are exact integers (<= 65280); one rounding at the end
// makes the result bit-identical to the direct 5 x 5 integer sum.
#include "vs_common.hpp"

namespace {

constexpr int TW = 128;                // output tile width
constexpr int TH = 32;                 // output tile height
constexpr int IH = 2 * TH + 3;
constexpr int OFF = 14;                // LDS byte offset of input column 2*x0-2 (16-byte aligned staging)
constexpr int LP = 288;                // LDS row pitch: OFF + IW rounded up to 16
constexpr int NCH = LP / 16;
constexpr int NLD = (NCH * IH + 255) / 256;
constexpr uint32_t RSRC_WORD3 = 0x00020000;   // raw (untyped) buffer access on gfx9-family parts
constexpr uint32_t W1464 = 0x04060401u;       // byte weights 1, 4, 6, 4 (byte 0 first)

__device__ __forceinline__ int refl101_clamped(int t, int n)
{
    if (t < 0) t = -t;
    if (t >= n) t = 2 * n - 2 - t;
    return vs::clampi(t, 0, n - 1);    // rows/columns only used by outputs past the edge
}

// item i of a strided call reads src + i * src_stride and writes dst + i * dst_stride
struct Strided {
    const uint8_t* src;
    int64_t src_stride;
    uint8_t* dst;
    int64_t dst_stride;
    __device__ __forceinline__ const uint8_t* in(int i) const { return src + i * src_stride; }
    __device__ __forceinline__ uint8_t* out(int i) const { return dst + i * dst_stride; }
};

// item i of a batched step: level l - 1 of the current frame's pyramid (level 0: the frame) to level l
struct Step {
    vs::StepView v;
    int64_t src_off, dst_off;
    int from_frame;
    __device__ __forceinline__ const uint8_t* in(int i) const
    {
        return from_frame ? v.frame(i, v.j(i)) : v.cur_pyr(i) + src_off;
    }
    __device__ __forceinline__ uint8_t* out(int i) const { return v.cur_pyr(i) + dst_off; }
};

template <class A>
__global__ __launch_bounds__(256) void pyr_down_kernel(A io, int src_pitch, int sw, int sh, int dst_pitch, int dw,
                                                        int dh, int n_items, int tiles_x, int tiles_y, int by_xcd,
                                                        int vec_ok)
{
    __shared__ __attribute__((aligned(16))) uint8_t tin[IH * LP];
    int item, tile;
    if (!vs::xcd_map(blockIdx.x, n_items, tiles_x * tiles_y, by_xcd != 0, item, tile)) return;
    const int ty = tile / tiles_x, tx = tile - ty * tiles_x;
    const uint8_t* s = io.in(item);
    uint8_t* d = io.out(item);
    const int ox = tx * TW, oy = ty * TH;
    const int ix0 = 2 * ox - 2, iy0 = 2 * oy - 2;
    const int tid = threadIdx.x;
    const int a0 = ix0 - OFF;                // global column of LDS byte 0 (may be negative)
    {
        using V4 = __attribute__((ext_vector_type(4))) unsigned int;
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t*>(s), (short)0,
                                                                            src_pitch * sh, RSRC_WORD3);
        // only input columns/rows that some output of the tile reads are staged: relative columns
        // [0, need_c) and rows [0, need_r); at the frame edges these reach 2 past it (reflect-101)
        const int need_c = 2 * min(TW, dw - ox) + 3, need_r = 2 * min(TH, dh - oy) + 3;
        V4 v[NLD];
#pragma unroll
        for (int j = 0; j < NLD; ++j) {
            const int k = tid + 256 * j;
            const int r = k / NCH, c = k - r * NCH;
            if (k < NCH * IH && r < need_r && 16 * c - OFF < need_c) {
                const int gy = refl101_clamped(iy0 + r, sh);
                const int gx = a0 + 16 * c;
                if (vec_ok && gx >= 0 && gx + 16 <= sw) {
                    v[j] = __builtin_bit_cast(V4, __builtin_amdgcn_raw_buffer_load_b128(rs, gy * src_pitch + gx, 0, 0));
                } else if (!vec_ok) {
                    // unaligned source rows: 16 byte loads from reflect-101 columns, issued together
                    uint32_t wd[4] = {0u, 0u, 0u, 0u};
#pragma unroll
                    for (int e = 0; e < 16; ++e) {
                        const uint32_t byte = __builtin_amdgcn_raw_buffer_load_b8(
                            rs, gy * src_pitch + refl101_clamped(gx + e, sw), 0, 0);
                        wd[e >> 2] |= byte << (8 * (e & 3));
                    }
                    v[j] = V4{wd[0], wd[1], wd[2], wd[3]};
                } else {
                    // chunk crossing an edge: its in-frame bytes (the reflected columns are filled in LDS)
                    uint32_t wd[4] = {0u, 0u, 0u, 0u};
#pragma unroll
                    for (int e = 0; e < 16; ++e) {
                        const int x = gx + e;
                        if (x >= 0 && x < sw)
                            wd[e >> 2] |= (uint32_t)__builtin_amdgcn_raw_buffer_load_b8(rs, gy * src_pitch + x, 0, 0)
                                          << (8 * (e & 3));
                    }
                    v[j] = V4{wd[0], wd[1], wd[2], wd[3]};
                }
            } else if (k < NCH * IH) {
                v[j] = V4{0u, 0u, 0u, 0u};
            }
        }
#pragma unroll
        for (int j = 0; j < NLD; ++j) {
            const int k = tid + 256 * j;
            const int r = k / NCH, c = k - r * NCH;
            if (k < NCH * IH && r < need_r && 16 * c - OFF < need_c)
                *reinterpret_cast<V4*>(&tin[16 * k]) = v[j];   // row r, chunk c at r * LP + 16 c
        }
        // reflect-101 columns: global column g sits at LDS byte OFF + g - ix0 of its row; left of the
        // frame -1, -2 mirror 1, 2; right of it sw, sw + 1 mirror sw - 2, sw - 3
        const bool left = ix0 < 0, right = ix0 + need_c > sw;
        if (vec_ok && (left || right)) {
            __syncthreads();
            if (tid < need_r) {
                uint8_t* row = &tin[tid * LP + OFF - ix0];
                if (left) {
                    row[-1] = row[1];
                    row[-2] = row[2];
                }
                if (right) {
                    row[sw] = row[sw - 2];
                    if (ix0 + need_c > sw + 1) row[sw + 1] = row[sw - 3];
                }
            }
        }
    }
    __syncthreads();

    const int g = tid & 31, rg = tid >> 5;     // 4 output columns 4g.., 4 output rows 4rg..
    const int x = ox + 4 * g, y = oy + 4 * rg;
    if (x >= dw || y >= dh) return;
    // input columns (relative to 2*ox-2) 8g .. 8g+10 sit at LDS bytes OFF+8g ..; the words read start
    // at OFF-2+8g (4-aligned) and hold relative columns 8g-2 .. 8g+13
    const uint32_t* wrow = reinterpret_cast<const uint32_t*>(&tin[(8 * rg) * LP + OFF - 2 + 8 * g]);
    uint32_t h[11][4];
#pragma unroll
    for (int j = 0; j < 11; ++j) {
        const uint32_t* w = wrow + j * (LP / 4);
        const uint32_t d0 = w[0], d1 = w[1], d2 = w[2], d3 = w[3];
        // d0 = cols -2..1, d1 = 2..5, d2 = 6..9, d3 = 10..13 (relative to 8g)
        const uint32_t a01 = __builtin_amdgcn_alignbyte(d1, d0, 2);   // cols 0..3
        const uint32_t a12 = __builtin_amdgcn_alignbyte(d2, d1, 2);   // cols 4..7
        h[j][0] = __builtin_amdgcn_udot4(d1, 0x00010000u, __builtin_amdgcn_udot4(a01, W1464, 0, false), false);
        h[j][1] = __builtin_amdgcn_udot4(d2, 0x00000001u, __builtin_amdgcn_udot4(d1, W1464, 0, false), false);
        h[j][2] = __builtin_amdgcn_udot4(d2, 0x00010000u, __builtin_amdgcn_udot4(a12, W1464, 0, false), false);
        h[j][3] = __builtin_amdgcn_udot4(d3, 0x00000001u, __builtin_amdgcn_udot4(d2, W1464, 0, false), false);
    }
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        if (y + m >= dh) break;
        uint32_t packed = 0;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const uint32_t t = h[2 * m][c] + h[2 * m + 4][c] + 128u + 4u * (h[2 * m + 1][c] + h[2 * m + 3][c]) +
                               6u * h[2 * m + 2][c];
            packed |= (t >> 8) << (8 * c);
        }
        uint8_t* out = d + (int64_t)(y + m) * dst_pitch + x;
        if (x + 4 <= dw && (dst_pitch & 3) == 0 && (reinterpret_cast<uintptr_t>(out) & 3) == 0)
            *reinterpret_cast<uint32_t*>(out) = packed;
        else
            for (int c = 0; c < 4 && x + c < dw; ++c) out[c] = (uint8_t)(packed >> (8 * c));
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
    if ((int64_t)layout->pitch[0] * layout->height[0] >= ((int64_t)1 << 31))
        return vs::set_error(VS_ERR_UNSUPPORTED, "vs_build_pyramid: frame larger than 2 GiB");
    hipStream_t s = vs::as_stream(stream);
    const bool by_xcd = n >= vs::xcd_min_items(vs::XCD_PYRAMID);
    for (int l = 1; l < layout->levels; ++l) {
        const uint8_t* src = (l == 1) ? frames : pyrs + layout->offset[l - 1];
        const int64_t sstride = (l == 1) ? frame_stride : pyr_stride;
        const int spitch = layout->pitch[l - 1];
        const int dw = layout->width[l], dh = layout->height[l];
        const int tiles_x = (dw + TW - 1) / TW, tiles_y = (dh + TH - 1) / TH;
        // 16-byte staging loads need 16-byte aligned rows in every item
        const bool vec_ok = (spitch % 16 == 0) && (reinterpret_cast<uintptr_t>(src) % 16 == 0) &&
                            (n == 1 || sstride % 16 == 0);
        const int64_t nblk = vs::xcd_grid(n, tiles_x * tiles_y, by_xcd);
        const Strided io{src, sstride, pyrs + layout->offset[l], pyr_stride};
        pyr_down_kernel<<<(unsigned)nblk, 256, 0, s>>>(io, spitch, layout->width[l - 1], layout->height[l - 1],
                                                       layout->pitch[l], dw, dh, n, tiles_x, tiles_y, by_xcd, vec_ok);
        int e = vs::check_launch("vs_build_pyramid");
        if (e) return e;
    }
    return VS_OK;
}

namespace vs {

// levels 1..L-1 of the current frame of every item of a batched step
int step_pyramid(const StepView& v, int n, const vs_pyramid& L, bool vec_ok, hipStream_t s)
{
    if (n <= 0 || L.levels == 1) return VS_OK;
    const bool by_xcd = n >= xcd_min_items(XCD_PYRAMID);
    for (int l = 1; l < L.levels; ++l) {
        const int dw = L.width[l], dh = L.height[l];
        const int tiles_x = (dw + TW - 1) / TW, tiles_y = (dh + TH - 1) / TH;
        const Step io{v, l == 1 ? 0 : L.offset[l - 1], L.offset[l], l == 1 ? 1 : 0};
        const int64_t nblk = xcd_grid(n, tiles_x * tiles_y, by_xcd);
        pyr_down_kernel<<<(unsigned)nblk, 256, 0, s>>>(io, L.pitch[l - 1], L.width[l - 1], L.height[l - 1], L.pitch[l],
                                                       dw, dh, n, tiles_x, tiles_y, by_xcd, (l == 1 ? vec_ok : true));
        const int e = check_launch("vs_batch_push(pyramid)");
        if (e) return e;
    }
    return VS_OK;
}

}  // namespace vs
