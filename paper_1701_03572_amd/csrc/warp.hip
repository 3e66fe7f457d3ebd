// warp_frame: inverse-mapped bilinear warp of 8-bit frames, all items of a batch in one launch.
//
// A 256-thread workgroup covers a 256 x 64 output tile (tall tiles spread the per-tile matrix
// inversion, source box and staging over more pixels). Wave w takes the tile's columns
// 64 w .. 64 w + 63; its lanes cover 64 columns x 4 rows at a time (4 consecutive pixels per lane,
// 16 lanes per row), and each thread produces its 4 pixels in 16 rows 4 apart, stored as one 32-bit
// word per row when the row allows it. The 2x3 matrix is
// inverted in binary64; per-pixel source coordinates are FP32, relative to the tile's source box.
//
// Source box: the map is affine and is evaluated in a form that is monotone in x and in y, so the
// extreme source coordinates of the tile's in-frame pixels are at its four corners. The box (plus a
// one-pixel margin) is staged in LDS with 16-byte loads; bytes outside the frame are staged as the
// border value, which gives every tap exactly the border semantics of a per-tap test. Each pixel then
// reads its four taps as single bytes from LDS (a fixed row pitch makes the lower taps immediate
// offsets; at 80 words it puts the four rows one instruction reads on distinct banks). Tiles whose box does not fit the LDS buffer (strong zoom-out or rotation) take a
// per-pixel path that reads the frame directly.
// Values are rounded half up: floor(v + 0.5) is an integer in [0, 255], packed exactly.
#include "vs_common.hpp"

namespace {

constexpr int TW = 256;                 // tile width: 4 waves x 16 lanes x 4 pixels
constexpr int RPT = 16;                 // rows per thread
constexpr int TH = 4 * RPT;             // 4 lane rows per wave
constexpr int LW = 320;                 // LDS row pitch (80 words: 16 mod 32 banks)
constexpr int BW = 288;                 // staged box width: 18 chunks of 16 bytes
constexpr int NCH = BW / 16;
constexpr int MAXR = 96;                // staged rows at most
constexpr int NLD = (NCH * MAXR + 255) / 256;
constexpr float BIG = 1048576.0f;       // boxes beyond +-2^20 take the direct path
constexpr uint32_t RSRC_WORD3 = 0x00020000;   // raw (untyped) buffer access on gfx9-family parts

__device__ __forceinline__ float lerp(float u, float v, float t) { return fmaf(t, v - u, u); }

struct Box {
    float mnx, mxx, mny, mxy;
    bool finite;   // every corner coordinate is a number inside (-2^20, 2^20)
};

// source-coordinate box of the pixels [ox, xe] x [oy, ye] under x' = f00 x + f01 y + c0, y' = f10 x + f11 y + c1,
// evaluated exactly as the per-pixel loop evaluates it
__device__ __forceinline__ Box corner_box(float f00, float f01, float c0, float f10, float f11, float c1, int ox, int xe,
                                          int oy, int ye)
{
    Box b{INFINITY, -INFINITY, INFINITY, -INFINITY, true};
#pragma unroll
    for (int cy = 0; cy < 2; ++cy)
#pragma unroll
        for (int cx = 0; cx < 2; ++cx) {
            const float fx = (float)(cx ? xe : ox), fy = (float)(cy ? ye : oy);
            const float sx = fmaf(f00, fx, fmaf(f01, fy, c0));
            const float sy = fmaf(f10, fx, fmaf(f11, fy, c1));
            b.mnx = fminf(b.mnx, sx);
            b.mxx = fmaxf(b.mxx, sx);
            b.mny = fminf(b.mny, sy);
            b.mxy = fmaxf(b.mxy, sy);
            b.finite = b.finite && sx > -BIG && sx < BIG && sy > -BIG && sy < BIG;   // false for NaN
        }
    return b;
}

// item i of a strided call: src + i * src_stride, matrix mats + i * mat_stride, dst + i * dst_stride
struct Strided {
    const uint8_t* src;
    int64_t src_stride;
    const double* mats;
    int64_t mat_stride;
    uint8_t* dst;
    int64_t dst_stride;
    __device__ __forceinline__ bool at(int i, const uint8_t*& s, const double*& M, uint8_t*& d) const
    {
        s = src + i * src_stride;
        M = mats + i * mat_stride;
        d = dst + i * dst_stride;
        return true;
    }
};

// item i of a batched step: the frame e = j - lag it emits (none while j < lag) under the matrix the
// smoother's step just wrote to mats[0], into output slot e % out_slots
struct Step {
    vs::StepView v;
    __device__ __forceinline__ bool at(int i, const uint8_t*& s, const double*& M, uint8_t*& d) const
    {
        const vs::StepStream& q = v.s(i);
        const int64_t e = q.next_frame - v.lag;
        if (e < 0) return false;
        s = v.frame(i, e);
        M = q.mats;
        d = q.out + (e % q.out_slots) * v.plane;
        return true;
    }
};

// 5 workgroups per CU: the LDS tile (96 rows of 288 bytes) allows no more
template <class IO>
__global__ __launch_bounds__(256, 5) void warp_kernel(IO io, int W, int H, int src_pitch, int dst_pitch, int border,
                                                      int tiles_x, int tiles_y, int vec_ok, int n_items, int by_xcd)
{
    __shared__ __attribute__((aligned(16))) uint8_t tin[MAXR * LW];
    // the tiles of one frame run on one XCD, so the halo rows of vertically adjacent tiles are
    // shared in its L2
    int item, tile;
    if (!vs::xcd_map(blockIdx.x, n_items, tiles_x * tiles_y, by_xcd != 0, item, tile)) return;
    const int ty = tile / tiles_x, tx = tile - ty * tiles_x;
    const int ox = tx * TW, oy = ty * TH;
    const int x4 = ox + 64 * (int)(threadIdx.x >> 6) + 4 * (int)(threadIdx.x & 15);
    const int ybase = oy + (int)((threadIdx.x >> 4) & 3);   // the thread's rows: ybase + 4 r
    const uint8_t* s;
    const double* M;
    uint8_t* dst;
    if (!io.at(item, s, M, dst)) return;
    // the item is the workgroup's: its pointers are uniform (a batched step reads them from memory)
    s = vs::uniform_ptr(s);
    M = vs::uniform_ptr(M);
    dst = vs::uniform_ptr(dst);
    const double rdet = 1.0 / (M[0] * M[4] - M[1] * M[3]);
    const double i00 = M[4] * rdet, i01 = -M[1] * rdet, i10 = -M[3] * rdet, i11 = M[0] * rdet;
    const double i02 = -(i00 * M[2] + i01 * M[5]);
    const double i12 = -(i10 * M[2] + i11 * M[5]);
    const float f00 = (float)i00, f01 = (float)i01;
    const float f10 = (float)i10, f11 = (float)i11;
    const int nx = W - x4 < 4 ? W - x4 : 4;      // <= 0 for threads past the right edge
    const int ny = H - ybase <= 0 ? 0 : ((H - ybase + 3) >> 2 < RPT ? (H - ybase + 3) >> 2 : RPT);
    uint8_t* drow = dst + (int64_t)ybase * dst_pitch + x4;
    const bool word_store = nx == 4 && (reinterpret_cast<uintptr_t>(drow) & 3) == 0 && (dst_pitch & 3) == 0;
    const int xe = (ox + TW < W ? ox + TW : W) - 1, ye = (oy + TH < H ? oy + TH : H) - 1;

    // box in absolute coordinates -> origin of the staged box (one pixel of margin on the low sides)
    const Box ab = corner_box(f00, f01, (float)i02, f10, f11, (float)i12, ox, xe, oy, ye);
    bool staged = ab.finite;
    int a0 = 0, by0 = 0, nr = 0;
    float g02 = 0.0f, g12 = 0.0f;
    if (staged) {
        a0 = ((int)floorf(ab.mnx) - 1) & ~15;
        by0 = (int)floorf(ab.mny) - 1;
        g02 = (float)(i02 - (double)a0);
        g12 = (float)(i12 - (double)by0);
        // the same box in the relative coordinates the pixels use: every tap must be inside the buffer
        const Box rb = corner_box(f00, f01, g02, f10, f11, g12, ox, xe, oy, ye);
        nr = (int)floorf(rb.mxy) + 2;
        staged = rb.finite && rb.mnx >= 0.0f && rb.mny >= 0.0f && rb.mxx < (float)(BW - 1) && nr <= MAXR;
    }
    if (staged) {
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t*>(s), (short)0,
                                                                            src_pitch * H, RSRC_WORD3);
        using V4 = __attribute__((ext_vector_type(4))) unsigned int;
        const uint32_t bw = (uint32_t)border * 0x01010101u;
        const int total = NCH * nr;
        V4 v[NLD];
#pragma unroll
        for (int j = 0; j < NLD; ++j) {
            const int k = threadIdx.x + 256 * j;
            v[j] = V4{bw, bw, bw, bw};
            if (k < total) {
                const int r = k / NCH, c = k - r * NCH;
                const int gy = by0 + r, gx = a0 + 16 * c;
                const bool row_in = gy >= 0 && gy < H;
                if (vec_ok && row_in && gx >= 0 && gx + 16 <= W) {
                    v[j] = __builtin_bit_cast(V4, __builtin_amdgcn_raw_buffer_load_b128(rs, gy * src_pitch + gx, 0, 0));
                } else if (row_in && gx < W && gx + 16 > 0) {
                    // chunk straddling the left or right edge (or an unaligned source): byte by byte
                    uint32_t wd[4] = {bw, bw, bw, bw};
                    for (int e = 0; e < 16; ++e) {
                        const int x = gx + e;
                        if (x >= 0 && x < W) {
                            const uint32_t byte = s[(int64_t)gy * src_pitch + x];
                            const int sh = 8 * (e & 3);
                            wd[e >> 2] = (wd[e >> 2] & ~(0xffu << sh)) | (byte << sh);
                        }
                    }
                    v[j] = V4{wd[0], wd[1], wd[2], wd[3]};
                }
            }
        }
#pragma unroll
        for (int j = 0; j < NLD; ++j) {
            const int k = threadIdx.x + 256 * j;
            if (k < total) {
                const int r = k / NCH, c = k - r * NCH;
                *reinterpret_cast<V4*>(&tin[r * LW + 16 * c]) = v[j];
            }
        }
        __syncthreads();
        if (nx <= 0 || ny <= 0) return;
        float fxq[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) fxq[q] = (float)(x4 + (q < nx ? q : nx - 1));   // past-the-edge columns repeat
        for (int r = 0; r < ny; ++r) {
            const float fy = (float)(ybase + 4 * r);
            const float bx = fmaf(f01, fy, g02), by = fmaf(f11, fy, g12);
            uint32_t packed = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float sx = fmaf(f00, fxq[q], bx);
                const float sy = fmaf(f10, fxq[q], by);
                const float x0 = floorf(sx), y0 = floorf(sy);
                const float a = sx - x0, b = sy - y0;
                const int p = (int)fmaf(y0, (float)LW, x0);   // exact: < 2^24
                int p1 = p + 1;
                // an empty asm hides that p1 = p + 1, so the taps stay single-byte reads (a merged 16-bit
                // read at an odd address takes the LDS unaligned path)
                asm volatile("" : "+v"(p1));
                const float v00 = (float)tin[p], v10 = (float)tin[p1];
                const float v01 = (float)tin[p + LW], v11 = (float)tin[p1 + LW];
                const float v = lerp(lerp(v00, v10, a), lerp(v01, v11, a), b);
                packed = __builtin_amdgcn_cvt_pk_u8_f32(floorf(v + 0.5f), q, packed);
            }
            uint8_t* out = drow + (int64_t)(4 * r) * dst_pitch;
            if (word_store) *reinterpret_cast<uint32_t*>(out) = packed;
            else
                for (int q = 0; q < nx; ++q) out[q] = (uint8_t)(packed >> (8 * q));
        }
        return;
    }
    if (nx <= 0 || ny <= 0) return;

    const float f02 = (float)i02, f12 = (float)i12;
    const float bord = (float)border;
    const float fW = (float)W, fH = (float)H;
    for (int r = 0; r < ny; ++r) {
        const float fy = (float)(ybase + 4 * r);
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
        uint8_t* out = drow + (int64_t)(4 * r) * dst_pitch;
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
    const bool by_xcd = n >= vs::xcd_min_items(vs::XCD_WARP);
    const int64_t nblk = vs::xcd_grid(n, tiles_x * tiles_y, by_xcd);
    if (nblk > 0x7fffffff) return vs::set_error(VS_ERR_INVALID, "vs_warp_frame: grid too large");
    // 16-byte staging loads need 16-byte aligned rows in every item
    const int vec_ok = (src_pitch % 16 == 0) && (reinterpret_cast<uintptr_t>(src) % 16 == 0) &&
                       (n == 1 || src_stride % 16 == 0);
    const Strided io{src, src_stride, mats, mat_stride, dst, dst_stride};
    warp_kernel<<<(unsigned)nblk, 256, 0, vs::as_stream(stream)>>>(io, width, height, src_pitch, dst_pitch, border,
                                                                   tiles_x, tiles_y, vec_ok, n, by_xcd);
    return vs::check_launch("vs_warp_frame");
}

namespace vs {

// the warp of the frame each item of a batched step emits (items emitting nothing return at once)
int step_warp(const StepView& v, int n, int W, int H, int border, bool vec_ok, hipStream_t s)
{
    if (n <= 0) return VS_OK;
    const int tiles_x = (W + TW - 1) / TW, tiles_y = (H + TH - 1) / TH;
    const bool by_xcd = n >= xcd_min_items(XCD_WARP);
    const int64_t nblk = xcd_grid(n, tiles_x * tiles_y, by_xcd);
    if (nblk > 0x7fffffff) return set_error(VS_ERR_INVALID, "vs_batch_push: warp grid too large");
    warp_kernel<<<(unsigned)nblk, 256, 0, s>>>(Step{v}, W, H, W, W, border, tiles_x, tiles_y, vec_ok ? 1 : 0, n, by_xcd);
    return check_launch("vs_batch_push(warp)");
}

}  // namespace vs
