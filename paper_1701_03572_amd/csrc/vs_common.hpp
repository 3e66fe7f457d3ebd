// Internal helpers shared by the HIP translation units of libvstab (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstring>

#include "vstab.h"

namespace vs {

// Records a message for vs_last_error() and returns `code`.
int set_error(int code, const char* fmt, ...);

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Checks the launch that was just enqueued.
int check_launch(const char* what);

// Launch tuning in force (vs_set_tuning): batches of at least xcd_min_items(k) items use the
// per-XCD mapping for kernel family k; tracking workgroups hold lk_points_per_group() points.
enum { XCD_PYRAMID = 0, XCD_LK = 1, XCD_WARP = 2 };
int xcd_min_items(int kernel);
int lk_points_per_group();

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Wave64 butterfly sum: every lane ends with the same, bit-identical total (each stage adds the
// same two operands in every lane, and addition is commutative).
__device__ __forceinline__ float wave_sum(float v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

__device__ __forceinline__ double wave_sum_d(double v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

__device__ __forceinline__ int wave_sum_i(int v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

// Wave64 sum through DPP: quad_perm [1,0,3,2], quad_perm [2,3,0,1], row_half_mirror and
// row_mirror leave every lane of a 16-lane row holding that row's sum (each step adds the same
// two operands in every lane, so the bits agree across the row); the four row sums are then read
// as uniform values and added in a fixed order. Every lane returns the identical total.
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, true));
}

// DPP move into the rows selected by ROW_MASK; the other rows receive 0.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_rows(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, ROW_MASK, 0xF,
                                                                 false));
}

// Two wave64 sums at once, steps interleaved: row sums by DPP as in wave_total, then
// row_bcast:15 into rows 1 and 3 and row_bcast:31 into rows 2 and 3 leave the total in lane 63,
// which is read as a uniform value (fixed order: (r0 + r1) + (r2 + r3)).
__device__ __forceinline__ void wave_total2(float& a, float& b)
{
    a += dpp_mov<0xB1>(a);
    b += dpp_mov<0xB1>(b);
    a += dpp_mov<0x4E>(a);
    b += dpp_mov<0x4E>(b);
    a += dpp_mov<0x141>(a);
    b += dpp_mov<0x141>(b);
    a += dpp_mov<0x140>(a);
    b += dpp_mov<0x140>(b);
    a += dpp_rows<0x142, 0xA>(a);
    b += dpp_rows<0x142, 0xA>(b);
    a += dpp_rows<0x143, 0xC>(a);
    b += dpp_rows<0x143, 0xC>(b);
    a = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, a), 63));
    b = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, b), 63));
}

__device__ __forceinline__ float wave_total(float v)
{
    v += dpp_mov<0xB1>(v);
    v += dpp_mov<0x4E>(v);
    v += dpp_mov<0x141>(v);
    v += dpp_mov<0x140>(v);
    v += dpp_rows<0x142, 0xA>(v);
    v += dpp_rows<0x143, 0xC>(v);
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
}

// Workgroup -> (item, tile) mapping of a one-dimensional grid. With `by_xcd`, the tiles of item i
// all run on the same XCD (workgroups are dealt to the 8 XCDs round-robin, so workgroup b runs on
// XCD b % 8): item i takes XCD i % 8 and its tiles are consecutive there, so neighbouring tiles
// share that XCD's L2. The grid then has 8 * ceil(n / 8) * tiles workgroups; the padding ones
// return at once.
__device__ __forceinline__ bool xcd_map(int b, int n_items, int tiles, bool by_xcd, int& item, int& tile)
{
    if (!by_xcd) {
        item = b / tiles;
        tile = b - item * tiles;
    } else {
        const int x = b & 7, k = b >> 3;
        const int q = k / tiles;
        tile = k - q * tiles;
        item = q * 8 + x;
    }
    return item < n_items;
}

// batches of at least this many items use the per-XCD mapping
#ifndef VS_XCD_MIN_ITEMS
#define VS_XCD_MIN_ITEMS 8
#endif

inline int64_t xcd_grid(int n_items, int tiles, bool by_xcd)
{
    return by_xcd ? (int64_t)8 * ((n_items + 7) / 8) * tiles : (int64_t)n_items * tiles;
}

struct LevelDesc {
    int32_t w[VS_MAX_LEVELS];
    int32_t h[VS_MAX_LEVELS];
    int32_t pitch[VS_MAX_LEVELS];
    int64_t off[VS_MAX_LEVELS];
    int32_t levels;
};

inline LevelDesc level_desc(const vs_pyramid& p)
{
    LevelDesc d{};
    d.levels = p.levels;
    for (int l = 0; l < VS_MAX_LEVELS; ++l) {
        d.w[l] = p.width[l];
        d.h[l] = p.height[l];
        d.pitch[l] = p.pitch[l];
        d.off[l] = p.offset[l];
    }
    return d;
}

}  // namespace vs
