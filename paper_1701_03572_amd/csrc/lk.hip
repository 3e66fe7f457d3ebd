// track_lk: pyramidal Lucas-Kanade with the forward-backward check, one wave64 per point slot.
//
// Lane layout for a (2h+1)^2 window: the window's 2h+1 columns are spread over the lanes and the
// rows over G = 64 / (2h+1) lane groups, each group owning R = ceil((2h+1) / G) consecutive rows
// (h = 10: 21 columns x 3 groups of 7 rows = 63 lanes). Every sample of the window shares one
// fractional offset, so a lane reads its (R+3) x 4 pixel block once per level, keeps I, dI/dx,
// dI/dy of its R samples in registers, and per iteration reads an (R+1) x 2 block of the next
// image. The three tensor sums and the two residual sums are wave butterfly reductions, whose
// totals are bit-identical in every lane, so the iteration control is wave-uniform.
#include "vs_common.hpp"

namespace {

struct Img {
    const uint8_t* p;
    int w, h, pitch;
};

__device__ __forceinline__ Img level_img(const uint8_t* frame, const uint8_t* pyr, const vs::LevelDesc& d, int l)
{
    Img im;
    im.p = (l == 0) ? frame : pyr + d.off[l];
    im.w = d.w[l];
    im.h = d.h[l];
    im.pitch = d.pitch[l];
    return im;
}

__device__ __forceinline__ float px(const Img& im, int x, int y)
{
    x = vs::clampi(x, 0, im.w - 1);
    y = vs::clampi(y, 0, im.h - 1);
    return (float)im.p[(int64_t)y * im.pitch + x];
}

__device__ __forceinline__ float bil(float a, float b, float v00, float v10, float v01, float v11)
{
    return (1.0f - b) * ((1.0f - a) * v00 + a * v10) + b * ((1.0f - a) * v01 + a * v11);
}

// g11 g22 - g12^2 with Kahan's compensated 2x2 determinant (one fma recovers the product error)
__device__ __forceinline__ float det2(float g11, float g22, float g12)
{
    const float w = g12 * g12;
    const float e = fmaf(-g12, g12, w);
    const float f = fmaf(g11, g22, -w);
    return f + e;
}

struct LKConst {
    int hw, cols, groups, rows, nwin;
    int max_iter;
    float eps2, min_eig;
};

template <int RMAX>
__device__ bool track_one(const uint8_t* fa, const uint8_t* pa, const uint8_t* fb, const uint8_t* pb,
                          const vs::LevelDesc& d, const LKConst& c, float ux, float uy, float& vx, float& vy,
                          uint32_t& n_setup, uint32_t& n_iter)
{
    const int lane = threadIdx.x & 63;
    const int gcol = lane % c.cols, grp = lane / c.cols;
    const bool active = grp < c.groups;
    const int qx = gcol - c.hw;
    const int qy0 = grp * c.rows - c.hw;                 // first window row of this lane
    int nrows = c.hw - qy0 + 1;                          // rows of this lane inside the window
    nrows = active ? (nrows < c.rows ? nrows : c.rows) : 0;
    nrows = nrows < 0 ? 0 : nrows;

    float gx = 0.f, gy = 0.f;
    bool ok = true;
    for (int l = d.levels - 1; l >= 0; --l) {
        const Img A = level_img(fa, pa, d, l);
        const Img B = level_img(fb, pb, d, l);
        const float sc = ldexpf(1.0f, -l);
        const float cx = ux * sc, cy = uy * sc;
        const float fx = floorf(cx), fy = floorf(cy);
        const float a = cx - fx, b = cy - fy;
        const int ix = (int)fx + qx, iy = (int)fy + qy0;

        float I[RMAX], Ix[RMAX], Iy[RMAX];
        float g11 = 0.f, g12 = 0.f, g22 = 0.f;
        {
            // rows iy-1 .. iy+nrows+1, columns ix-1 .. ix+2
            float p0[4], p1[4], p2[4], p3[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                p0[t] = px(A, ix - 1 + t, iy - 1);
                p1[t] = px(A, ix - 1 + t, iy);
                p2[t] = px(A, ix - 1 + t, iy + 1);
            }
#pragma unroll
            for (int k = 0; k < RMAX; ++k) {
                if (k < nrows) {
#pragma unroll
                    for (int t = 0; t < 4; ++t) p3[t] = px(A, ix - 1 + t, iy + k + 2);
                    // p0: row k-1, p1: row k, p2: row k+1, p3: row k+2 (relative to iy)
                    I[k] = bil(a, b, p1[1], p1[2], p2[1], p2[2]);
                    Ix[k] = 0.5f * bil(a, b, p1[2] - p1[0], p1[3] - p1[1], p2[2] - p2[0], p2[3] - p2[1]);
                    Iy[k] = 0.5f * bil(a, b, p2[1] - p0[1], p2[2] - p0[2], p3[1] - p1[1], p3[2] - p1[2]);
                    g11 += Ix[k] * Ix[k];
                    g12 += Ix[k] * Iy[k];
                    g22 += Iy[k] * Iy[k];
#pragma unroll
                    for (int t = 0; t < 4; ++t) { p0[t] = p1[t]; p1[t] = p2[t]; p2[t] = p3[t]; }
                } else {
                    I[k] = Ix[k] = Iy[k] = 0.f;
                }
            }
        }
        g11 = vs::wave_sum(g11);
        g12 = vs::wave_sum(g12);
        g22 = vs::wave_sum(g22);
        ++n_setup;
        const float tr = g11 + g22;
        const float s = sqrtf((g11 - g22) * (g11 - g22) + 4.0f * g12 * g12);
        const float lmax = 0.5f * (tr + s);
        const float det = det2(g11, g22, g12);
        const float lmin = lmax > 0.f ? det / lmax : 0.f;
        float nux = 0.f, nuy = 0.f;
        if (!(lmin / (float)c.nwin >= c.min_eig)) {
            if (l == 0) ok = false;
        } else {
            const float inv = 1.0f / det;
            for (int it = 0; it < c.max_iter; ++it) {
                const float pxx = cx + gx + nux, pyy = cy + gy + nuy;
                const float jfx = floorf(pxx), jfy = floorf(pyy);
                const float ja = pxx - jfx, jb = pyy - jfy;
                const int jx = (int)jfx + qx, jy = (int)jfy + qy0;
                float b1 = 0.f, b2 = 0.f;
                if (nrows > 0) {
                    float q0a = px(B, jx, jy), q0b = px(B, jx + 1, jy);
#pragma unroll
                    for (int k = 0; k < RMAX; ++k) {
                        if (k < nrows) {
                            const float q1a = px(B, jx, jy + k + 1), q1b = px(B, jx + 1, jy + k + 1);
                            const float J = bil(ja, jb, q0a, q0b, q1a, q1b);
                            const float dlt = I[k] - J;
                            b1 += dlt * Ix[k];
                            b2 += dlt * Iy[k];
                            q0a = q1a;
                            q0b = q1b;
                        }
                    }
                }
                b1 = vs::wave_sum(b1);
                b2 = vs::wave_sum(b2);
                const float ex = (g22 * b1 - g12 * b2) * inv;
                const float ey = (g11 * b2 - g12 * b1) * inv;
                nux += ex;
                nuy += ey;
                ++n_iter;
                if (ex * ex + ey * ey < c.eps2) break;
            }
        }
        if (l > 0) {
            gx = 2.0f * (gx + nux);
            gy = 2.0f * (gy + nuy);
        } else {
            vx = ux + gx + nux;
            vy = uy + gy + nuy;
        }
    }
    if (!(vx >= 0.f && vy >= 0.f && vx <= (float)(d.w[0] - 1) && vy <= (float)(d.h[0] - 1))) ok = false;
    return ok;
}

template <int RMAX>
__global__ __launch_bounds__(256) void lk_kernel(const uint8_t* __restrict__ prev_frames,
                                                 const uint8_t* __restrict__ prev_pyrs,
                                                 const uint8_t* __restrict__ next_frames,
                                                 const uint8_t* __restrict__ next_pyrs, int64_t frame_stride,
                                                 int64_t pyr_stride, int istride, vs::LevelDesc d,
                                                 const float* xy_prev, const uint8_t* alive_prev, int capacity,
                                                 LKConst c, int fb, float fb_thresh, float* xy_next, uint8_t* status,
                                                 float* fb_err, int32_t* n_valid, float* xy_chain,
                                                 uint8_t* alive_chain, unsigned long long* work)
{
    const int slot = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int item = blockIdx.y;
    if (slot >= capacity) return;
    const int lane = threadIdx.x & 63;
    const int64_t rec = (int64_t)item * istride;
    const int64_t k = rec * capacity + slot;
    const float ux = xy_prev[2 * k], uy = xy_prev[2 * k + 1];
    const bool alive = alive_prev ? alive_prev[k] != 0 : true;
    float vx = ux, vy = uy, err = __int_as_float(0x7fc00000);
    bool ok = false;
    uint32_t n_setup = 0, n_iter = 0;
    if (alive) {
        const uint8_t* fa = prev_frames + item * frame_stride;
        const uint8_t* pa = prev_pyrs + item * pyr_stride;
        const uint8_t* fb_ = next_frames + item * frame_stride;
        const uint8_t* pb = next_pyrs + item * pyr_stride;
        ok = track_one<RMAX>(fa, pa, fb_, pb, d, c, ux, uy, vx, vy, n_setup, n_iter);
        if (ok && fb) {
            float bx = vx, by = vy;
            const bool okb = track_one<RMAX>(fb_, pb, fa, pa, d, c, vx, vy, bx, by, n_setup, n_iter);
            err = sqrtf((bx - ux) * (bx - ux) + (by - uy) * (by - uy));
            ok = okb && err <= fb_thresh;
        }
    }
    if (lane == 0) {
        xy_next[2 * k] = vx;
        xy_next[2 * k + 1] = vy;
        status[k] = ok ? 1 : 0;
        if (fb_err) fb_err[k] = err;
        if (xy_chain) {
            xy_chain[2 * k] = vx;
            xy_chain[2 * k + 1] = vy;
        }
        if (alive_chain) alive_chain[k] = ok ? 1 : 0;
        if (ok && n_valid) atomicAdd(&n_valid[rec], 1);
        if (work && n_setup) {
            atomicAdd(&work[0], (unsigned long long)n_setup);
            atomicAdd(&work[1], (unsigned long long)n_iter);
        }
    }
}

__global__ void zero_counters(int32_t* p, int n, int istride, unsigned long long* work)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (p && i < n) p[(int64_t)i * istride] = 0;
    if (work && i < 2) work[i] = 0;
}

}  // namespace

extern "C" int vs_track_lk(const uint8_t* prev_frames, const uint8_t* prev_pyrs, const uint8_t* next_frames,
                           const uint8_t* next_pyrs, int64_t frame_stride, int64_t pyr_stride, int32_t n,
                           int32_t istride, const vs_pyramid* layout, const float* xy_prev, const uint8_t* alive_prev, int32_t capacity,
                           const vs_lk_params* p, float* xy_next, uint8_t* status, float* fb_err, int32_t* n_valid,
                           float* xy_chain, uint8_t* alive_chain, uint64_t* work, void* stream)
{
    if (!layout || !p) return vs::set_error(VS_ERR_INVALID, "vs_track_lk: null argument");
    if (n < 0 || capacity < 0 || istride < 1) return vs::set_error(VS_ERR_INVALID, "vs_track_lk: negative count");
    if (n == 0 || capacity == 0) return VS_OK;
    if (!prev_frames || !next_frames || !xy_prev || !xy_next || !status)
        return vs::set_error(VS_ERR_INVALID, "vs_track_lk: null argument");
    if (layout->levels > 1 && (!prev_pyrs || !next_pyrs))
        return vs::set_error(VS_ERR_INVALID, "vs_track_lk: null pyramid");
    if (layout->levels < 1 || layout->levels > VS_MAX_LEVELS)
        return vs::set_error(VS_ERR_UNSUPPORTED, "vs_track_lk: levels out of range");
    if (capacity > VS_MAX_CORNERS) return vs::set_error(VS_ERR_UNSUPPORTED, "vs_track_lk: capacity > %d", VS_MAX_CORNERS);
    if (p->win_half < 1 || p->win_half > 15) return vs::set_error(VS_ERR_UNSUPPORTED, "vs_track_lk: win_half must be 1..15");
    if (p->max_iter < 1 || !(p->eps >= 0.f) || !(p->min_eig >= 0.f) || !(p->fb_thresh >= 0.f))
        return vs::set_error(VS_ERR_INVALID, "vs_track_lk: bad parameters");
    if (n > 65535) return vs::set_error(VS_ERR_INVALID, "vs_track_lk: more than 65535 items");
    LKConst c;
    c.hw = p->win_half;
    c.cols = 2 * c.hw + 1;
    c.groups = 64 / c.cols;
    c.rows = (c.cols + c.groups - 1) / c.groups;
    c.nwin = c.cols * c.cols;
    c.max_iter = p->max_iter;
    c.eps2 = p->eps * p->eps;
    c.min_eig = p->min_eig;
    hipStream_t s = vs::as_stream(stream);
    unsigned long long* wk = reinterpret_cast<unsigned long long*>(work);
    if (n_valid || wk) {
        zero_counters<<<(n + 255) / 256, 256, 0, s>>>(n_valid, n, istride, wk);
        int e = vs::check_launch("vs_track_lk(zero)");
        if (e) return e;
    }
    const vs::LevelDesc d = vs::level_desc(*layout);
    dim3 grid((capacity + 3) / 4, n);
    if (c.rows <= 7)
        lk_kernel<7><<<grid, 256, 0, s>>>(prev_frames, prev_pyrs, next_frames, next_pyrs, frame_stride, pyr_stride,
                                          istride, d, xy_prev, alive_prev, capacity, c, p->fb, p->fb_thresh, xy_next,
                                          status, fb_err, n_valid, xy_chain, alive_chain, wk);
    else
        lk_kernel<16><<<grid, 256, 0, s>>>(prev_frames, prev_pyrs, next_frames, next_pyrs, frame_stride, pyr_stride,
                                           istride, d, xy_prev, alive_prev, capacity, c, p->fb, p->fb_thresh, xy_next,
                                           status, fb_err, n_valid, xy_chain, alive_chain, wk);
    return vs::check_launch("vs_track_lk");
}
