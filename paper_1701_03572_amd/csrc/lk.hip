// track_lk: pyramidal Lucas-Kanade with the forward-backward check, one wave64 (one workgroup)
// per point slot.
//
// Lane layout for a (2h+1)^2 window: the window's 2h+1 columns are spread over the lanes and the
// rows over G = 64 / (2h+1) lane groups, each group owning R = ceil((2h+1) / G) consecutive rows
// (h = 10: 21 columns x 3 groups of 7 rows = 63 lanes). Samples outside the window get zero
// gradient weight, so every lane runs the same branch-free loops. All samples of a window share
// one fractional offset, so per level a lane reads its (R+3) x 4 previous-frame block once (one
// unaligned 32-bit load per row when the whole window is inside the level, edge-clamped byte loads
// otherwise), interpolates each row horizontally first and derives I, dI/dx, dI/dy of its R samples
// into registers.
//
// Gauss-Newton iterations: all samples also share the iterate's fractional offset (ja, jb), so the
// residual sum over the window, sum (I - J) grad I, is E0 - ja E1 - jb E2 - ja jb E3 with four sums
// per gradient component that depend only on the iterate's integer position (the bilinear form of
// the next-frame 2 x 2 blocks; see residual_partials). They are recomputed, from the lane's (R+1) x 2
// next-frame block, only when the integer position moves; an iteration that stays on the same
// pixel costs a few wave-uniform operations. The lanes accumulate plain sums of products of raw
// next-frame pixels with the gradients (no per-sample differences), and the E sums are formed from
// the reduced totals. The first block of each level is read with the set-up, and its eight sums
// share the set-up's reduction with the three tensor sums and the two sums of I times the gradient. Reductions are
// transposing DPP row sums, so several sums cost little more than one; every lane ends with the
// same totals, and the iteration control is wave-uniform. One wave per workgroup lets every point
// retire independently.
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

__device__ __forceinline__ bool wave_all(bool c) { return __ballot(!c) == 0; }

// Next-frame 2-pixel rows x0, x0 + 1 of rows y0 .. y0 + RMAX: qa = P(x0), qb = P(x0 + 1). When every
// active lane's block is inside the level, one (unaligned) 16-bit load per row; otherwise
// edge-clamped byte loads.
template <int RMAX>
__device__ __forceinline__ void load_next_block(const Img& B, int x0, int y0, bool active, float (&qa)[RMAX + 1],
                                                float (&qb)[RMAX + 1])
{
    const bool b_in = wave_all(!active || (x0 >= 0 && x0 + 1 <= B.w - 1 && y0 >= 0 && y0 + RMAX <= B.h - 1));
    if (b_in) {
#pragma unroll
        for (int k = 0; k <= RMAX; ++k) {
            const uint32_t w = __builtin_amdgcn_raw_buffer_load_b16(
                B.rs, (int)__umul24((unsigned)(y0 + k), (unsigned)B.pitch) + x0, 0, 0);
            qa[k] = (float)(w & 0xff);
            qb[k] = (float)((w >> 8) & 0xff);
        }
    } else {
        const int c0 = vs::clampi(x0, 0, B.w - 1), c1 = vs::clampi(x0 + 1, 0, B.w - 1);
#pragma unroll
        for (int k = 0; k <= RMAX; ++k) {
            const int base = (int)__umul24((unsigned)vs::clampi(y0 + k, 0, B.h - 1), (unsigned)B.pitch);
            qa[k] = ld(B, base + c0);
            qb[k] = ld(B, base + c1);
        }
    }
}

// Lane partials of the residual sums for the next-frame block (qa, qb) at integer offset (x0, y0).
// With the iterate's fraction (ja, jb), the bilinear next-frame sample of window pixel k is
// P00 + ja d10 + jb d01 + ja jb d11 with P00 = qa_k, d10 = qb_k - qa_k, d01 = qa_{k+1} - qa_k and
// d11 = (qb_{k+1} - qa_{k+1}) - (qb_k - qa_k), so
//   sum_k (I_k - J_k) Ix_k = E0x - ja E1x - jb E2x - ja jb E3x,
// with, from the plain sums A0 = sum qa_k Ix_k, A1 = sum qa_{k+1} Ix_k, B0 = sum qb_k Ix_k,
// B1 = sum qb_{k+1} Ix_k and S = sum I_k Ix_k:
//   E0x = S - A0, E1x = B0 - A0, E2x = A1 - A0, E3x = (B1 - A1) - (B0 - A0)
// (likewise for Iy). The sums depend on the integer offset only. Output order:
// A0x A1x B0x B1x A0y A1y B0y B1y.
template <int RMAX>
__device__ __forceinline__ void residual_partials(const float (&Ix)[RMAX], const float (&Iy)[RMAX],
                                                  const float (&qa)[RMAX + 1], const float (&qb)[RMAX + 1], float* e)
{
#pragma unroll
    for (int j = 0; j < 8; ++j) e[j] = 0.f;
#pragma unroll
    for (int k = 0; k < RMAX; ++k) {
        e[0] = fmaf(qa[k], Ix[k], e[0]);
        e[1] = fmaf(qa[k + 1], Ix[k], e[1]);
        e[2] = fmaf(qb[k], Ix[k], e[2]);
        e[3] = fmaf(qb[k + 1], Ix[k], e[3]);
        e[4] = fmaf(qa[k], Iy[k], e[4]);
        e[5] = fmaf(qa[k + 1], Iy[k], e[5]);
        e[6] = fmaf(qb[k], Iy[k], e[6]);
        e[7] = fmaf(qb[k + 1], Iy[k], e[7]);
    }
}

// E sums of one gradient component from its reduced plain sums (see residual_partials)
__device__ __forceinline__ void e_from_sums(float S, float A0, float A1, float B0, float B1, float* E)
{
    E[0] = S - A0;
    E[1] = B0 - A0;
    E[2] = A1 - A0;
    E[3] = (B1 - A1) - (B0 - A0);
}

// Previous-frame samples of one lane: I, and the gradient terms 0.5 * central differences (zero
// outside the window), at rows iy .. iy + RMAX - 1 and column ix, offset by the shared fraction (a, b).
// Rows iy-1 .. iy+RMAX+1 and columns ix-1 .. ix+2 are read: with FAST (every lane's block inside the
// level) one unaligned 32-bit load per row, otherwise four edge-clamped byte loads. Rows are
// interpolated horizontally first.
template <int RMAX, bool FAST>
__device__ __forceinline__ void window_samples(const Img& A, int ix, int iy, float a, float b, int nrows, float (&I)[RMAX],
                                               float (&Ix)[RMAX], float (&Iy)[RMAX])
{
    float H1[RMAX + 3], Dd[RMAX + 3];   // per row: horizontal lerp at the sample column, and the
                                        // horizontal central difference lerped the same way
#pragma unroll
    for (int r = 0; r < RMAX + 3; ++r) {
        float p0, p1, p2, p3;
        if constexpr (FAST) {
            const uint32_t w = __builtin_amdgcn_raw_buffer_load_b32(
                A.rs, (int)__umul24((unsigned)(iy - 1 + r), (unsigned)A.pitch) + ix - 1, 0, 0);
            p0 = (float)(w & 0xff);
            p1 = (float)((w >> 8) & 0xff);
            p2 = (float)((w >> 16) & 0xff);
            p3 = (float)(w >> 24);
        } else {
            const int base = (int)__umul24((unsigned)vs::clampi(iy - 1 + r, 0, A.h - 1), (unsigned)A.pitch);
            p0 = ld(A, base + vs::clampi(ix - 1, 0, A.w - 1));
            p1 = ld(A, base + vs::clampi(ix, 0, A.w - 1));
            p2 = ld(A, base + vs::clampi(ix + 1, 0, A.w - 1));
            p3 = ld(A, base + vs::clampi(ix + 2, 0, A.w - 1));
        }
        H1[r] = lerp(p1, p2, a);
        Dd[r] = lerp(p2, p3, a) - lerp(p0, p1, a);
    }
#pragma unroll
    for (int k = 0; k < RMAX; ++k) {
        // sample row k sits between rows k + 1 and k + 2
        const float wgt = k < nrows ? 0.5f : 0.0f;   // zero weight outside the window
        I[k] = lerp(H1[k + 1], H1[k + 2], b);
        Ix[k] = wgt * lerp(Dd[k + 1], Dd[k + 2], b);
        Iy[k] = wgt * lerp(H1[k + 2] - H1[k], H1[k + 3] - H1[k + 1], b);
    }
}

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

        // ---- window set-up: rows iy-1 .. iy+RMAX+1, columns ix-1 .. ix+2 of the previous frame. When
        // every lane's block is inside the level, a row is one (unaligned) 32-bit load; otherwise four
        // edge-clamped byte loads.
        const bool a_in = wave_all(!active || (ix - 1 >= 0 && ix + 2 <= A.w - 1 && iy - 1 >= 0 && iy + RMAX + 1 <= A.h - 1));
        float I[RMAX], Ix[RMAX], Iy[RMAX];
        if (a_in)
            window_samples<RMAX, true>(A, ix, iy, a, b, nrows, I, Ix, Iy);
        else
            window_samples<RMAX, false>(A, ix, iy, a, b, nrows, I, Ix, Iy);
        // the first iterate's next-frame block is read here, so its residual sums share the set-up's
        // reduction: 3 tensor sums + 2 sums of I times the gradient + 8 residual sums in one
        // transposing reduction
        int cjx = (int)floorf(cx + gx), cjy = (int)floorf(cy + gy);
        float qa[RMAX + 1], qb[RMAX + 1];
        load_next_block<RMAX>(B, cjx + qx, cjy + qy0, active, qa, qb);
        float v[16];
        residual_partials<RMAX>(Ix, Iy, qa, qb, v + 5);
        v[0] = v[1] = v[2] = v[3] = v[4] = 0.f;
#pragma unroll
        for (int k = 0; k < RMAX; ++k) {
            v[0] = fmaf(Ix[k], Ix[k], v[0]);
            v[1] = fmaf(Ix[k], Iy[k], v[1]);
            v[2] = fmaf(Iy[k], Iy[k], v[2]);
            v[3] = fmaf(I[k], Ix[k], v[3]);
            v[4] = fmaf(I[k], Iy[k], v[4]);
        }
#pragma unroll
        for (int j = 13; j < 16; ++j) v[j] = 0.f;
        const float tot = vs::wave_transpose_sum<16>(v);
        const float g11 = vs::transposed_total<16>(tot, 0), g12 = vs::transposed_total<16>(tot, 1);
        const float g22 = vs::transposed_total<16>(tot, 2);
        const float Sx = vs::transposed_total<16>(tot, 3), Sy = vs::transposed_total<16>(tot, 4);
        float E[8];
        e_from_sums(Sx, vs::transposed_total<16>(tot, 5), vs::transposed_total<16>(tot, 6),
                    vs::transposed_total<16>(tot, 7), vs::transposed_total<16>(tot, 8), E);
        e_from_sums(Sy, vs::transposed_total<16>(tot, 9), vs::transposed_total<16>(tot, 10),
                    vs::transposed_total<16>(tot, 11), vs::transposed_total<16>(tot, 12), E + 4);
        ++n_setup;
        const float tr = g11 + g22;
        const float sq = sqrtf((g11 - g22) * (g11 - g22) + 4.0f * g12 * g12);
        const float lmax = 0.5f * (tr + sq);
        const float det = det2(g11, g22, g12);
        const float lmin = lmax > 0.f ? det / lmax : 0.f;
        float nux = 0.f, nuy = 0.f;
        if (!(lmin / (float)c.nwin >= c.min_eig)) {
            if (l == 0) ok = false;
        } else {
            const float inv = __builtin_amdgcn_rcpf(det);
            for (int it = 0; it < c.max_iter; ++it) {
                const float pxx = cx + gx + nux, pyy = cy + gy + nuy;
                const float jfx = floorf(pxx), jfy = floorf(pyy);
                const float ja = pxx - jfx, jb = pyy - jfy;
                const int jx = (int)jfx, jy = (int)jfy;
                if (jx != cjx || jy != cjy) {
                    // the integer position moved: new block, new residual sums
                    cjx = jx;
                    cjy = jy;
                    load_next_block<RMAX>(B, jx + qx, jy + qy0, active, qa, qb);
                    float e[8];
                    residual_partials<RMAX>(Ix, Iy, qa, qb, e);
                    const float t8 = vs::wave_transpose_sum<8>(e);
                    e_from_sums(Sx, vs::transposed_total<8>(t8, 0), vs::transposed_total<8>(t8, 1),
                                vs::transposed_total<8>(t8, 2), vs::transposed_total<8>(t8, 3), E);
                    e_from_sums(Sy, vs::transposed_total<8>(t8, 4), vs::transposed_total<8>(t8, 5),
                                vs::transposed_total<8>(t8, 6), vs::transposed_total<8>(t8, 7), E + 4);
                }
                const float b1 = E[0] - fmaf(ja, fmaf(jb, E[3], E[1]), jb * E[2]);
                const float b2 = E[4] - fmaf(ja, fmaf(jb, E[7], E[5]), jb * E[6]);
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
                                                int64_t pyr_stride, int istride, vs::LevelDesc d, const float* xy_prev,
                                                const uint8_t* alive_prev, int capacity, LKConst c, int fb,
                                                float fb_thresh, float* xy_next, uint8_t* status, float* fb_err,
                                                int32_t* n_valid, float* xy_chain, uint8_t* alive_chain,
                                                unsigned long long* work, int n_items, int by_xcd)
{
    // each wave of the workgroup tracks one point slot on its own (no barriers): slot = group *
    // waves + wave. All point slots of an item run on one XCD, so the overlapping windows of its
    // frame pair are shared in that XCD's L2.
    const int ppg = blockDim.x >> 6;
    const int groups = (capacity + ppg - 1) / ppg;
    int item, group;
    if (!vs::xcd_map(blockIdx.x, n_items, groups, by_xcd != 0, item, group)) return;
    const int slot = group * ppg + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));   // wave-uniform
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
        if (work && n_setup) {   // per-item counters: one address per item keeps the atomics uncontended
            atomicAdd(&work[2 * item], (unsigned long long)n_setup);
            atomicAdd(&work[2 * item + 1], (unsigned long long)n_iter);
        }
    }
}

__global__ void zero_counters(int32_t* p, int n, int istride, unsigned long long* work)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (p && i < n) p[(int64_t)i * istride] = 0;
    if (work && i < n) {
        work[2 * i] = 0;
        work[2 * i + 1] = 0;
    }
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
    if ((int64_t)layout->pitch[0] * layout->height[0] >= ((int64_t)1 << 31) || layout->pitch[0] >= (1 << 24))
        return vs::set_error(VS_ERR_UNSUPPORTED, "vs_track_lk: frame larger than 2 GiB or rows of 16 MiB");
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
    const bool by_xcd = n >= vs::xcd_min_items(vs::XCD_LK);
    const int ppg = vs::lk_points_per_group();
    const int64_t nblk = vs::xcd_grid(n, (capacity + ppg - 1) / ppg, by_xcd);
    if (nblk > 0x7fffffff) return vs::set_error(VS_ERR_INVALID, "vs_track_lk: grid too large");
    const unsigned grid = (unsigned)nblk;
    const unsigned threads = 64u * (unsigned)ppg;
    if (c.rows <= 7)
        lk_kernel<7><<<grid, threads, 0, s>>>(prev_frames, prev_pyrs, next_frames, next_pyrs, frame_stride, pyr_stride,
                                         istride, d, xy_prev, alive_prev, capacity, c, p->fb, p->fb_thresh, xy_next,
                                         status, fb_err, n_valid, xy_chain, alive_chain, wk, n, by_xcd);
    else
        lk_kernel<16><<<grid, threads, 0, s>>>(prev_frames, prev_pyrs, next_frames, next_pyrs, frame_stride, pyr_stride,
                                          istride, d, xy_prev, alive_prev, capacity, c, p->fb, p->fb_thresh, xy_next,
                                          status, fb_err, n_valid, xy_chain, alive_chain, wk, n, by_xcd);
    return vs::check_launch("vs_track_lk");
}
