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
