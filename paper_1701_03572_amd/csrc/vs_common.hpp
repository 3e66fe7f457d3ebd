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
// rows per corner-response wave segment for a batch of n_items (few_rows / many_rows by default)
int detect_segment_rows(int n_items, int few_rows, int many_rows);
// hypothesis workgroups of a fit launch in flight
int fit_groups_in_flight();

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Orders one wave's LDS accesses across its lanes: LDS operations of a wave complete in issue order,
// and the fences keep the compiler from moving accesses across this point.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// A pointer every lane of the wave holds equally, as a scalar (a buffer descriptor made from it then
// stays in scalar registers instead of being re-checked lane by lane before every load).
template <class T>
__device__ __forceinline__ T* uniform_ptr(T* p)
{
    const uint64_t v = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return reinterpret_cast<T*>(((uint64_t)hi << 32) | lo);
}

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

// ------------------------------------------------------------------------------------------------
// Batched per-frame step (vs_batch_*): one launch per stage covers the current frame of every stream
// of a batch. Each attached stream has a device descriptor (its vs_stream buffers, the parameters that
// may differ between the streams of a batch, and a device-side frame counter); a step's items name
// descriptor slots. Every stage reads an item's frame index from its descriptor, so a step's launches
// are the same from one frame to the next (a captured step can be replayed).
struct StepStream {
    const uint8_t* ring;        // the stream's frames: frame j at ring + (j % ring_len) * plane
    uint8_t* pyr;               // two pyramids: frame j's at pyr + (j & 1) * pyr_bytes
    float* pts;                 // [2][capacity][2]: the points tracked from frame j at [j & 1]
    uint8_t* alive;             // [2][capacity]
    float* dst;                 // [capacity][2]
    uint8_t* status;            // [capacity]
    float* fb_err;              // [capacity]
    int32_t* n_valid;           // [1]
    int32_t* count;             // [1]
    vs_fit_state* fit_state;
    double* pair_params;        // [1][4]
    double* affine6;            // [1][6]
    vs_fit_info* info;          // [1]
    uint8_t* inliers;           // [capacity]
    void* traj_state;
    double* mats;               // [lag + 2][6]
    int32_t* n_emitted;
    int64_t* first_frame;
    uint8_t* out;               // [out_slots][plane]
    int64_t next_frame;         // the frame the next step processes (advanced on the device)
    int32_t ring_len;
    int32_t out_slots;
    int32_t max_corners;
    int32_t pad;
    uint64_t seed;
    int64_t stream_id;
};

// One step's view, passed by value to its kernels: item i is the stream of descriptor slot[i].
struct StepView {
    StepStream* desc;
    const int32_t* slot;        // device, [n]
    int64_t plane;              // frame bytes (pitch = width)
    int64_t pyr_bytes;
    int32_t capacity;           // point slots of every stream of the batch
    int32_t lag;                // the smoother's lag (frames)
    int32_t redetect_every;
    int32_t min_valid;

    __device__ __forceinline__ StepStream& s(int i) const { return desc[slot[i]]; }
    __device__ __forceinline__ int64_t j(int i) const { return desc[slot[i]].next_frame; }
    __device__ __forceinline__ const uint8_t* frame(int i, int64_t k) const
    {
        const StepStream& d = desc[slot[i]];
        return d.ring + (k % d.ring_len) * plane;
    }
    __device__ __forceinline__ uint8_t* cur_pyr(int i) const { return s(i).pyr + (j(i) & 1) * pyr_bytes; }
    __device__ __forceinline__ uint8_t* prev_pyr(int i) const { return s(i).pyr + ((j(i) + 1) & 1) * pyr_bytes; }
};

// Stage launchers of the batched step (each defined next to its kernels); items [0, n) of the view.
int step_pyramid(const StepView& v, int n, const vs_pyramid& L, bool vec_ok, hipStream_t s);
int step_track(const StepView& v, int n, const vs_pyramid& L, const vs_lk_params& p, hipStream_t s);
size_t step_fit_workspace(int n, int capacity);
int step_fit(const StepView& v, int n, const vs_fit_params& p, uint8_t* ws, hipStream_t s);
int step_smooth(const StepView& v, int n, const vs_smooth_params& p, hipStream_t s);
int step_warp(const StepView& v, int n, int W, int H, int border, bool vec_ok, hipStream_t s);
int step_detect(const StepView& v, int n, int W, int H, const vs_detect_params& p, uint8_t* ws, hipStream_t s);

}  // namespace vs
