// track_lk: pyramidal Lucas-Kanade with the forward-backward check, one wave64 (one workgroup)
// per point slot.
//
// Lane layout for a (2h+1)^2 window: the window's 2h+1 columns are spread over the lanes and the
// rows over G = 64 / (2h+1) lane groups, each group owning R = ceil((2h+1) / G) consecutive rows
// (h = 10: 21 columns x 3 groups of 7 rows = 63 lanes). Samples outside the window get zero
// gradient weight, so every lane runs the same branch-free loops. All samples of a window share
// one fractional offset, so per level a lane reads its (R+3) x 4 pixel block once (buffer loads
// with 32-bit offsets, edge-clamped), interpolates each row horizontally first and derives I,
// dI/dx, dI/dy of its R samples into registers. Each Gauss-Newton iteration needs the lane's
// (R+1) x 2 next-frame block; it stays in registers while the iterate's integer position is
// unchanged and is reloaded when it moves. The three tensor sums and the two residual sums are
// DPP row reductions plus four lane reads, giving every lane the same total, so the iteration
// control is wave-uniform. One wave per workgroup lets every point retire independently.
#include "vs_common.hpp"

namespace {

constexpr uint32_t RSRC_WORD3 = 0x00020000;   // raw (untyped) buffer access on gfx9-family parts

struct Img {
    __amdgpu_buffer_rsrc_t rs;
    int w, h, pitch;
};

__device__ __forceinline__ Img level_img(const uint8_t* frame, const uint8_t* pyr, const vs::LevelDesc& d, int l)
{
    Img im;
    const uint8_t* p = (l == 0) ? frame : pyr + d.off[l];
    im.w = d.w[l];
    im.h = d.h[l];
    im.pitch = d.pitch[l];
    // loads past the level's bytes would return 0; clamped coordinates never get there
    im.rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t*>(p), (short)0, im.pitch * im.h, RSRC_WORD3);
    return im;
}

__device__ __forceinline__ float ld(const Img& im, int off)
{
    return (float)__builtin_amdgcn_raw_buffer_load_b8(im.rs, off, 0, 0);
}

__device__ __forceinline__ float lerp(float u, float v, float t) { return fmaf(t, v - u, u); }

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

        // ---- window set-up: rows iy-1 .. iy+RMAX+1, columns ix-1 .. ix+2 of the previous frame
        int col[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) col[t] = vs::clampi(ix - 1 + t, 0, A.w - 1);
        float H1[4], Dd[4];             // sliding rows: horizontal lerp at the sample column, and
                                        // the horizontal central difference lerped the same way
        auto row_terms = [&](int r, float& h1, float& dd) {
            const int base = (int)__umul24((unsigned)vs::clampi(iy - 1 + r, 0, A.h - 1), (unsigned)A.pitch);
            const float p0 = ld(A, base + col[0]), p1 = ld(A, base + col[1]);
            const float p2 = ld(A, base + col[2]), p3 = ld(A, base + col[3]);
            h1 = lerp(p1, p2, a);
            dd = lerp(p2, p3, a) - lerp(p0, p1, a);
        };
        row_terms(0, H1[0], Dd[0]);
        row_terms(1, H1[1], Dd[1]);
        row_terms(2, H1[2], Dd[2]);
        float I[RMAX], Ix[RMAX], Iy[RMAX];
        float g11 = 0.f, g12 = 0.f, g22 = 0.f;
#pragma unroll
        for (int k = 0; k < RMAX; ++k) {
            row_terms(k + 3, H1[3], Dd[3]);
            // sample row k sits between sliding rows 1 and 2
            const float wgt = k < nrows ? 0.5f : 0.0f;   // zero weight outside the window
            I[k] = lerp(H1[1], H1[2], b);
            Ix[k] = wgt * lerp(Dd[1], Dd[2], b);
            Iy[k] = wgt * lerp(H1[2] - H1[0], H1[3] - H1[1], b);
            g11 = fmaf(Ix[k], Ix[k], g11);
            g12 = fmaf(Ix[k], Iy[k], g12);
            g22 = fmaf(Iy[k], Iy[k], g22);
            H1[0] = H1[1]; H1[1] = H1[2]; H1[2] = H1[3];
            Dd[0] = Dd[1]; Dd[1] = Dd[2]; Dd[2] = Dd[3];
        }
        vs::wave_total2(g11, g12);
        g22 = vs::wave_total(g22);
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
            const float inv = __builtin_amdgcn_rcpf(det);
            int cjx = 0x7fffffff, cjy = 0;                // cached integer position of the next block
            float qa[RMAX + 1], qd[RMAX + 1];             // next-frame column jx and (jx + 1) - jx
            for (int it = 0; it < c.max_iter; ++it) {
                const float pxx = cx + gx + nux, pyy = cy + gy + nuy;
                const float jfx = floorf(pxx), jfy = floorf(pyy);
                const float ja = pxx - jfx, jb = pyy - jfy;
                const int jx = (int)jfx, jy = (int)jfy;
                if (jx != cjx || jy != cjy) {
                    cjx = jx;
                    cjy = jy;
                    const int c0 = vs::clampi(jx + qx, 0, B.w - 1), c1 = vs::clampi(jx + qx + 1, 0, B.w - 1);
#pragma unroll
                    for (int k = 0; k <= RMAX; ++k) {
                        const int base = (int)__umul24((unsigned)vs::clampi(jy + qy0 + k, 0, B.h - 1), (unsigned)B.pitch);
                        qa[k] = ld(B, base + c0);
                        qd[k] = ld(B, base + c1) - qa[k];
                    }
                }
                float b1 = 0.f, b2 = 0.f;
                float h0 = fmaf(ja, qd[0], qa[0]);
#pragma unroll
                for (int k = 0; k < RMAX; ++k) {
                    const float h1 = fmaf(ja, qd[k + 1], qa[k + 1]);
                    const float dlt = I[k] - lerp(h0, h1, jb);
                    b1 = fmaf(dlt, Ix[k], b1);
                    b2 = fmaf(dlt, Iy[k], b2);
                    h0 = h1;
                }
                vs::wave_total2(b1, b2);
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
__global__ __launch_bounds__(64) void lk_kernel(const uint8_t* __restrict__ prev_frames,
                                                const uint8_t* __restrict__ prev_pyrs,
                                                const uint8_t* __restrict__ next_frames,
                                                const uint8_t* __restrict__ next_pyrs, int64_t frame_stride,
                                                int64_t pyr_stride, int istride, vs::LevelDesc d, const float* xy_prev,
                                                const uint8_t* alive_prev, int capacity, LKConst c, int fb,
                                                float fb_thresh, float* xy_next, uint8_t* status, float* fb_err,
                                                int32_t* n_valid, float* xy_chain, uint8_t* alive_chain,
                                                unsigned long long* work)
{
    const int slot = blockIdx.x;
    const int item = blockIdx.y;
    const int lane = threadIdx.x;
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
                           int32_t istride, const vs_pyramid* layout, const float* xy_prev, const uint8_t* alive_prev,
                           int32_t capacity, const vs_lk_params* p, float* xy_next, uint8_t* status, float* fb_err,
                           int32_t* n_valid, float* xy_chain, uint8_t* alive_chain, uint64_t* work, void* stream)
{
    if (!layout || !p) return vs::set_error(VS_ERR_INVALID, "vs_track_lk: null argument");
    if (n < 0 || capacity < 0 || istride < 1) return vs::set_error(VS_ERR_INVALID, "vs_track_lk: bad count or stride");
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
    if ((int64_t)layout->pitch[0] * layout->height[0] >= ((int64_t)1 << 31))
        return vs::set_error(VS_ERR_UNSUPPORTED, "vs_track_lk: frame larger than 2 GiB");
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
    dim3 grid(capacity, n);
    if (c.rows <= 7)
        lk_kernel<7><<<grid, 64, 0, s>>>(prev_frames, prev_pyrs, next_frames, next_pyrs, frame_stride, pyr_stride,
                                         istride, d, xy_prev, alive_prev, capacity, c, p->fb, p->fb_thresh, xy_next,
                                         status, fb_err, n_valid, xy_chain, alive_chain, wk);
    else
        lk_kernel<16><<<grid, 64, 0, s>>>(prev_frames, prev_pyrs, next_frames, next_pyrs, frame_stride, pyr_stride,
                                          istride, d, xy_prev, alive_prev, capacity, c, p->fb, p->fb_thresh, xy_next,
                                          status, fb_err, n_valid, xy_chain, alive_chain, wk);
    return vs::check_launch("vs_track_lk");
}
