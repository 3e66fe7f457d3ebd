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

// Wave64 butterfly sums: every lane ends with the same, bit-identical total (each stage adds the
// same two operands in every lane, and addition is commutative).
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
