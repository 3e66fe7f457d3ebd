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

// Transposing row sum of N = 8 or 16 values per lane. Each step pairs every lane with a partner that
// differs in one lane bit (row_mirror: bit 3, row_half_mirror: bit 2, quad_perm [2,3,0,1]: bit 1,
// quad_perm [1,0,3,2]: bit 0; each partner lies in the same half of the previous pairing); the lane
// keeps one half of its values, adds the partner's copy of that half and hands over the other half.
// On return lane L holds the sum over its 16-lane row of value (L & 15) for N = 16, or of value
// ((L >> 1) & 7) for N = 8. wave_transpose_sum then adds the four rows, so every lane holds the
// wave total of its value; value j is read as a uniform with transposed_total().
template <int CTRL, int BIT, int M, int N>
__device__ __forceinline__ void transpose_step(float (&v)[N], int lane)
{
    const bool up = (lane >> BIT) & 1;
#pragma unroll
    for (int j = 0; j < M / 2; ++j) {
        const float lo = v[j], hi = v[j + M / 2];
        const float send = up ? lo : hi, keep = up ? hi : lo;
        v[j] = keep + dpp_mov<CTRL>(send);
    }
}

template <int N>
__device__ __forceinline__ float wave_transpose_sum(float (&v)[N])
{
    static_assert(N == 8 || N == 16, "8 or 16 values");
    const int lane = threadIdx.x & 63;
    transpose_step<0x140, 3, N>(v, lane);        // row_mirror
    transpose_step<0x141, 2, N / 2>(v, lane);    // row_half_mirror
    transpose_step<0x4E, 1, N / 4>(v, lane);     // quad_perm [2,3,0,1]
    float t;
    if constexpr (N == 16) {
        transpose_step<0xB1, 0, 2>(v, lane);     // quad_perm [1,0,3,2]
        t = v[0];
    } else {
        t = v[0] + dpp_mov<0xB1>(v[0]);
    }
    t += __shfl_xor(t, 16, 64);
    t += __shfl_xor(t, 32, 64);
    return t;
}

// uniform read of value j of a wave_transpose_sum<N> result
template <int N>
__device__ __forceinline__ float transposed_total(float t, int j)
{
    const int src = (N == 16) ? j : 2 * j;
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, t), src));
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
