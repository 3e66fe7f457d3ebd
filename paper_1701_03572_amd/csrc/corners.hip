// detect_corners: Shi-Tomasi response + 3x3 NMS over the ROI, then the ordered greedy top-K.
//
// Kernel 1 (corner_response): each wave walks down a 240-column strip of the ROI, 60 output rows at a
// time; lane i owns 4 columns. Per pixel row it forms, in registers, the Sobel terms (byte dot
// products), the tensor products and their 3x3 box sums (exact int32), an FP32 estimate of the score
// with a bounded relative error, and a separable 3x3 max of the estimates; neighbouring lanes' edge
// columns arrive by DPP wave shifts. A pixel whose neighbours' estimates are all below its own by
// more than the error band survives; one whose neighbours are above by more than the band is
// dropped; a pixel inside the band survives flagged. Survivors are appended (one atomic per wave and
// row) as their exact box-summed tensor (A, B, C) and pixel index.
//
// Kernel 2 (corner_keys): one thread per appended survivor computes the exact binary64 score
// 2 det / (tr + sqrt(disc)) from exact det/tr/disc; a flagged survivor is compared exactly against
// its in-ROI neighbours, recomputed from the image. Survivors that remain are written, compacted, to
// the item's candidate list, and the item's maximum score is folded in with an integer atomic max on
// the score's bit pattern (non-negative doubles order like their bits). The result is exactly the
// set of 3x3 maxima of the exact scores.
//
// Kernel 3 (corner_select): one 1024-thread workgroup per item. Candidates below
// quality * max are dropped. The order is (score desc, y asc, x asc), i.e. the composite key
// V = (bits(score) - bits(threshold)) * 2^32 + (2^32 - 1 - y * W - x) taken descending. Batches of
// the next ~2048 keys are cut out by a most-significant-digit radix select (11-bit digits),
// bitonic-sorted in LDS and fed to the greedy minimum-distance test 64 at a time: all 16 waves
// test a group against the accepted set, then one wave resolves conflicts inside the group in
// order. The result equals the sequential greedy over the full sorted list.
#include "vs_common.hpp"

namespace {

typedef unsigned __int128 u128;

struct CandHeader {
    uint32_t count;        // candidates (exact 3x3 maxima) in the key/index lists
    uint32_t raw_count;    // survivor-list entries reserved by the response kernel (unused ones are marked)
    uint64_t lmax_bits;
};

constexpr int64_t HDR = 256;
constexpr int SW = 240;         // output columns per wave strip (lanes 1..62 of 64 x 4 columns)
constexpr int SUP = 6;          // rows per unrolled super-step (period of the register rotation)
constexpr int SR = 60;          // output rows per wave: the pipeline runs SR + 6 pixel rows
constexpr int SR_FEW = 12;      // rows per wave for batches of at most 8 frames (more waves per frame)
constexpr int CAP = 4096;       // LDS batch capacity of the selection
constexpr int BATCH = 2048;     // keys requested per batch
constexpr int DIGIT = 11;
constexpr int NBIN = 1 << DIGIT;
// Each response wave reserves its survivor-list entries RAW_CHUNK at a time (one atomic per chunk
// rather than one per row on the frame's single counter, whose atomics serialise in L2); entries
// of a chunk it does not fill are marked RAW_UNUSED.
constexpr uint32_t RAW_CHUNK = 256;   // >= 4 columns x 64 lanes, so one row's survivors always fit
constexpr uint32_t RAW_UNUSED = 0xFFFFFFFFu;

// response waves of one item at most (the smaller segment height, strips over the whole width)
__host__ __device__ inline int64_t max_waves(int w, int h) { return (int64_t)(w / SW + 2) * (h / SR_FEW + 2); }

// per item: header | keys (8 B each) | indices (4 B) | survivors (16 B: A, B, C, index | flag << 31);
// the key and index lists have room for one entry per pixel, the survivor list also for one
// partly filled chunk per response wave
__host__ __device__ inline int64_t raw_entries(int w, int h) { return (int64_t)w * h + max_waves(w, h) * RAW_CHUNK; }
__host__ __device__ inline int64_t per_item_bytes(int w, int h)
{
    const int64_t c = (int64_t)w * h;
    return (HDR + 8 * c + 4 * c + 16 * raw_entries(w, h) + 255) & ~(int64_t)255;
}

__device__ __forceinline__ CandHeader* hdr_of(uint8_t* ws, int64_t item_bytes, int item)
{
    return reinterpret_cast<CandHeader*>(ws + item * item_bytes);
}
__device__ __forceinline__ uint64_t* keys_of(uint8_t* ws, int64_t item_bytes, int item)
{
    return reinterpret_cast<uint64_t*>(ws + item * item_bytes + HDR);
}
__device__ __forceinline__ uint32_t* idx_of(uint8_t* ws, int64_t item_bytes, int item, int w, int h)
{
    return reinterpret_cast<uint32_t*>(ws + item * item_bytes + HDR + 8 * (int64_t)w * h);
}
__device__ __forceinline__ uint4* raw_of(uint8_t* ws, int64_t item_bytes, int item, int w, int h)
{
    return reinterpret_cast<uint4*>(ws + item * item_bytes + HDR + 12 * (int64_t)w * h);
}

// Item addressing of a strided call: item i reads frames + i * frame_stride and owns the records
// g = i * istride; it is skipped when gate[g] >= gate_min.
struct Strided {
    const uint8_t* frames;
    int64_t frame_stride;
    int istride;
    const int32_t* gate;
    int gate_min;
    const int32_t* k_items;
    int capacity;
    float* xy;
    double* score;
    int32_t* count;
    uint8_t* alive;
    __device__ __forceinline__ bool off(int i) const { return gate != nullptr && gate[(int64_t)i * istride] >= gate_min; }
    __device__ __forceinline__ const uint8_t* img(int i) const { return frames + i * frame_stride; }
    __device__ __forceinline__ int budget(int i, int Kmax) const
    {
        if (!k_items) return Kmax;
        const int k = k_items[i];
        return k < 0 ? 0 : (k < Kmax ? k : Kmax);
    }
    __device__ __forceinline__ int64_t rec(int i) const { return (int64_t)i * istride; }
    __device__ __forceinline__ float* xy_of(int i) const { return xy + rec(i) * capacity * 2; }
    __device__ __forceinline__ double* score_of(int i) const { return score ? score + rec(i) * capacity : nullptr; }
    __device__ __forceinline__ int32_t* count_of(int i) const { return count + rec(i); }
    __device__ __forceinline__ uint8_t* alive_of(int i) const { return alive + rec(i) * capacity; }
};

// Item addressing of a batched step: frame j of the item's stream, detected on at j = 0 and every
// redetect_every frames, otherwise only when the pair just tracked has fewer than min_valid valid
// points; the corners go to the stream's point record [j & 1] (the points tracked from frame j).
struct Step {
    vs::StepView v;
    __device__ __forceinline__ bool off(int i) const
    {
        const vs::StepStream& d = v.s(i);
        const int64_t j = d.next_frame;
        return j != 0 && j % v.redetect_every != 0 && *d.n_valid >= v.min_valid;
    }
    __device__ __forceinline__ const uint8_t* img(int i) const { return v.frame(i, v.j(i)); }
    __device__ __forceinline__ int budget(int i, int Kmax) const
    {
        const int k = v.s(i).max_corners;
        return k < 0 ? 0 : (k < Kmax ? k : Kmax);
    }
    __device__ __forceinline__ int cur(int i) const { return (int)(v.j(i) & 1); }
    __device__ __forceinline__ float* xy_of(int i) const { return v.s(i).pts + (int64_t)cur(i) * v.capacity * 2; }
    __device__ __forceinline__ double* score_of(int) const { return nullptr; }
    __device__ __forceinline__ int32_t* count_of(int i) const { return v.s(i).count; }
    __device__ __forceinline__ uint8_t* alive_of(int i) const { return v.s(i).alive + (int64_t)cur(i) * v.capacity; }
};

template <class IO>
__global__ void detect_init_kernel(uint8_t* ws, int64_t item_bytes, int n, IO io)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || io.off(i)) return;
    CandHeader* h = hdr_of(ws, item_bytes, i);
    h->count = 0;
    h->raw_count = 0;
    h->lmax_bits = 0;
}

// Exact binary64 score 2 det / (tr + sqrt(disc)) of the box-summed tensor. With |A|, |B|, |C| < 2^24
// every product and sum below is an integer below 2^53, so det, tr and disc are exact and equal
// to their 64-bit integer values; sqrt, add and divide are single correctly rounded operations.
__device__ __forceinline__ double exact_key(int32_t A, int32_t B, int32_t C)
{
    const double a = (double)A, b = (double)B, c = (double)C;
    const double det = a * c - b * b;
    const double tr = a + c;
    const double dm = a - c;
    const double disc = dm * dm + 4.0 * (b * b);
    if (tr == 0.0) return 0.0;
    return __ddiv_rn(2.0 * det, __dadd_rn(tr, __dsqrt_rn(disc)));
}

// FP32 estimate of the same score. A, B and C are integers below 2^24 in magnitude, so they are
// exact floats. det comes from Kahan's compensated 2x2 determinant (relative error at most 2u,
// u = 2^-24, hence the exact sign, and 0 exactly when det == 0); disc = (A - C)^2 + 4 fl(B^2) is one
// fused rounding over non-negative terms (A - C is exact); with the sum A + C, the square root and
// the reciprocal (each within one ulp) and the final product the relative error stays below 10u
// (6e-7).
__device__ __forceinline__ float approx_key(int32_t A, int32_t B, int32_t C)
{
    const float a = (float)A, b = (float)B, c = (float)C;
    const float w = b * b;
    const float e = fmaf(-b, b, w);        // w - b^2, exactly
    const float det = fmaf(a, c, -w) + e;
    if (!(det > 0.0f)) return 0.0f;
    const float dm = a - c;
    const float disc = fmaf(dm, dm, 4.0f * w);
    const float sf = __builtin_amdgcn_sqrtf(disc);
    return 2.0f * det * __builtin_amdgcn_rcpf((a + c) + sf);
}

// half-width of the band inside which two FP32 estimates are compared exactly
constexpr float KEY_BAND = 1e-5f;

// exact box-summed Sobel tensor at (x, y) from the image (all pixels within 2 of (x, y) are read)
__device__ void tensor_from_image(const uint8_t* img, int pitch, int x, int y, int32_t& A, int32_t& B, int32_t& C)
{
    A = B = C = 0;
    for (int by = -1; by <= 1; ++by)
        for (int bx = -1; bx <= 1; ++bx) {
            const uint8_t* r0 = img + (int64_t)(y + by - 1) * pitch + (x + bx);
            const uint8_t* r1 = r0 + pitch;
            const uint8_t* r2 = r1 + pitch;
            const int gx = (r0[1] - r0[-1]) + 2 * (r1[1] - r1[-1]) + (r2[1] - r2[-1]);
            const int gy = (r2[-1] - r0[-1]) + 2 * (r2[0] - r0[0]) + (r2[1] - r0[1]);
            A += gx * gx;
            B += gx * gy;
            C += gy * gy;
        }
}

constexpr int DPP_SHR = 0x138;   // wave_shr:1 -- lane i receives lane i-1
constexpr int DPP_SHL = 0x130;   // wave_shl:1 -- lane i receives lane i+1

template <int CTRL>
__device__ __forceinline__ int dpp_i(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}

// Register state of one lane's 4 columns, indexed by pixel-row step modulo 3 (horizontal Sobel terms,
// horizontal box sums of the products, 3x3 maxima of the estimates) or modulo 2 (box sums, estimates,
// side maxima). All indices are compile-time constants after unrolling.
struct RespState {
    int dx[3][4], sy[3][4];
    int ha[3][4], hb[3][4], hc[3][4];
    int sa[2][4], sb[2][4], sc[2][4];
    float sv[2][4], hm[3][4], sd[2][4];
    uint32_t cbase, cfill;   // the wave's current survivor chunk (wave-uniform) and its fill
};

// marks entries [from, to) of the survivor list unused (the whole wave writes them)
__device__ __forceinline__ void mark_unused(uint4* raw, uint32_t from, uint32_t to, int lane)
{
    for (uint32_t i = from + lane; i < to; i += 64) raw[i] = make_uint4(0u, 0u, 0u, RAW_UNUSED);
}

struct RespCtx {
    int lane, xb, oy, oy_end;
    int rx0, rx1, ry0, ry1;
    int out_lo, out_hi;          // output columns of this strip
    int W;
    uint32_t* raw_count;
    uint4* raw;
};

// One pixel-row step. T is the step number modulo SUP; GRAD/BOX/NMS switch the pipeline stages on.
// Pixel row yp = oy - 3 + t; gradients for row yp - 1; box sums and estimates for row yp - 2; NMS
// decisions for row yp - 3.
template <int T, bool GRAD, bool BOX, bool NMS>
__device__ __forceinline__ void resp_step(RespState& st, uint32_t P, int t, const RespCtx& cx)
{
    constexpr int i3 = T % 3, m3 = (T + 2) % 3, mm3 = (T + 1) % 3;   // t, t-1, t-2 (mod 3)
    constexpr int i2 = T % 2, m2 = (T + 1) % 2;                       // t, t-1 (mod 2)
    const uint32_t L = (uint32_t)dpp_i<DPP_SHR>((int)P), R = (uint32_t)dpp_i<DPP_SHL>((int)P);
    // horizontal Sobel terms: (1,2,1) smoothing and central difference
    st.sy[i3][0] = (int)__builtin_amdgcn_udot4(L, 0x01000000u, __builtin_amdgcn_udot4(P, 0x00000102u, 0, false), false);
    st.sy[i3][1] = (int)__builtin_amdgcn_udot4(P, 0x00010201u, 0, false);
    st.sy[i3][2] = (int)__builtin_amdgcn_udot4(P, 0x01020100u, 0, false);
    st.sy[i3][3] = (int)__builtin_amdgcn_udot4(R, 0x00000001u, __builtin_amdgcn_udot4(P, 0x02010000u, 0, false), false);
    const int b0 = (int)(P & 0xff), b1 = (int)((P >> 8) & 0xff), b2 = (int)((P >> 16) & 0xff), b3 = (int)(P >> 24);
    st.dx[i3][0] = b1 - (int)(L >> 24);
    st.dx[i3][1] = b2 - b0;
    st.dx[i3][2] = b3 - b1;
    st.dx[i3][3] = (int)(R & 0xff) - b2;
    if constexpr (GRAD) {
        int A[4], B[4], C[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int gx = st.dx[mm3][c] + 2 * st.dx[m3][c] + st.dx[i3][c];
            const int gy = st.sy[i3][c] - st.sy[mm3][c];
            A[c] = __mul24(gx, gx);
            B[c] = __mul24(gx, gy);
            C[c] = __mul24(gy, gy);
        }
        const int al = dpp_i<DPP_SHR>(A[3]), ar = dpp_i<DPP_SHL>(A[0]);
        const int bl = dpp_i<DPP_SHR>(B[3]), br = dpp_i<DPP_SHL>(B[0]);
        const int cl = dpp_i<DPP_SHR>(C[3]), cr = dpp_i<DPP_SHL>(C[0]);
        st.ha[i3][0] = al + A[0] + A[1];
        st.hb[i3][0] = bl + B[0] + B[1];
        st.hc[i3][0] = cl + C[0] + C[1];
#pragma unroll
        for (int c = 1; c < 3; ++c) {
            st.ha[i3][c] = A[c - 1] + A[c] + A[c + 1];
            st.hb[i3][c] = B[c - 1] + B[c] + B[c + 1];
            st.hc[i3][c] = C[c - 1] + C[c] + C[c + 1];
        }
        st.ha[i3][3] = A[2] + A[3] + ar;
        st.hb[i3][3] = B[2] + B[3] + br;
        st.hc[i3][3] = C[2] + C[3] + cr;
    }
    if constexpr (BOX) {
        const int yb = cx.oy - 5 + t;
        const bool row_in = yb >= cx.ry0 && yb < cx.ry1;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            st.sa[i2][c] = st.ha[mm3][c] + st.ha[m3][c] + st.ha[i3][c];
            st.sb[i2][c] = st.hb[mm3][c] + st.hb[m3][c] + st.hb[i3][c];
            st.sc[i2][c] = st.hc[mm3][c] + st.hc[m3][c] + st.hc[i3][c];
            const int x = cx.xb + c;
            const bool in = row_in && x >= cx.rx0 && x < cx.rx1;
            st.sv[i2][c] = in ? approx_key(st.sa[i2][c], st.sb[i2][c], st.sc[i2][c]) : -1.0f;   // -1: ignored
        }
        const float sl = dpp_f<DPP_SHR>(st.sv[i2][3]), sr = dpp_f<DPP_SHL>(st.sv[i2][0]);
        st.hm[i3][0] = fmaxf(fmaxf(sl, st.sv[i2][0]), st.sv[i2][1]);
        st.sd[i2][0] = fmaxf(sl, st.sv[i2][1]);
#pragma unroll
        for (int c = 1; c < 3; ++c) {
            st.hm[i3][c] = fmaxf(fmaxf(st.sv[i2][c - 1], st.sv[i2][c]), st.sv[i2][c + 1]);
            st.sd[i2][c] = fmaxf(st.sv[i2][c - 1], st.sv[i2][c + 1]);
        }
        st.hm[i3][3] = fmaxf(fmaxf(st.sv[i2][2], st.sv[i2][3]), sr);
        st.sd[i2][3] = fmaxf(st.sv[i2][2], sr);
    }
    if constexpr (NMS) {
        const int yn = cx.oy - 6 + t;
        const bool row_ok = yn < cx.oy_end;
        bool surv[4], flag[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const float v = st.sv[m2][c];
            const float nmax = fmaxf(fmaxf(st.hm[mm3][c], st.hm[i3][c]), st.sd[m2][c]);
            const int x = cx.xb + c;
            const bool ok = row_ok && cx.lane >= 1 && cx.lane <= 62 && x >= cx.out_lo && x < cx.out_hi && v > 0.0f;
            surv[c] = ok && !(nmax > v * (1.0f + KEY_BAND));
            flag[c] = !(nmax < v * (1.0f - KEY_BAND));
        }
        uint64_t bal[4];
        uint32_t tot = 0;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            bal[c] = __ballot(surv[c]);
            tot += (uint32_t)__popcll(bal[c]);
        }
        if (tot) {
            if (st.cfill + tot > RAW_CHUNK) {
                // the current chunk is full: mark its rest unused and reserve the next one
                if (st.cbase != RAW_UNUSED) mark_unused(cx.raw, st.cbase + st.cfill, st.cbase + RAW_CHUNK, cx.lane);
                uint32_t b = 0;
                if (cx.lane == 0) b = atomicAdd(cx.raw_count, RAW_CHUNK);
                st.cbase = (uint32_t)__builtin_amdgcn_readfirstlane((int)b);
                st.cfill = 0;
            }
            uint32_t base = st.cbase + st.cfill;
            st.cfill += tot;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const uint32_t lo = (uint32_t)bal[c], hi = (uint32_t)(bal[c] >> 32);
                const uint32_t pos = base + __builtin_amdgcn_mbcnt_hi(hi, __builtin_amdgcn_mbcnt_lo(lo, 0u));
                if (surv[c]) {
                    const uint32_t ix = (uint32_t)(yn * cx.W + cx.xb + c) | (flag[c] ? 0x80000000u : 0u);
                    cx.raw[pos] = make_uint4((uint32_t)st.sa[m2][c], (uint32_t)st.sb[m2][c], (uint32_t)st.sc[m2][c], ix);
                }
                base += (uint32_t)__popcll(bal[c]);
            }
        }
    }
}

template <class IO>
__global__ __launch_bounds__(256) void corner_response_kernel(IO io, int W, int H, int pitch, int mx, int my, int n_items,
                                                              int strips, int segs, int sr, uint8_t* ws,
                                                              int64_t item_bytes)
{
    const int gw = blockIdx.x * 4 + (threadIdx.x >> 6);   // one independent wave per (item, strip, segment)
    const int per_item = strips * segs;
    const int item = gw / per_item;
    if (item >= n_items) return;
    if (io.off(item)) return;
    const int rem = gw - item * per_item;
    const int seg = rem / strips, strip = rem - seg * strips;

    RespCtx cx;
    cx.lane = threadIdx.x & 63;
    cx.W = W;
    cx.rx0 = mx; cx.rx1 = W - mx; cx.ry0 = my; cx.ry1 = H - my;
    cx.out_lo = mx + SW * strip;
    cx.out_hi = min(cx.out_lo + SW, cx.rx1);
    cx.xb = ((cx.out_lo - 4) & ~3) + 4 * cx.lane;   // lanes 1..62 cover [out_lo, out_lo + SW)
    cx.oy = my + sr * seg;
    cx.oy_end = min(cx.oy + sr, cx.ry1);
    cx.raw_count = &hdr_of(ws, item_bytes, item)->raw_count;
    cx.raw = raw_of(ws, item_bytes, item, W, H);   // room for raw_entries(W, H) entries

    // pixel rows are read through a buffer descriptor: rows or columns past the image read as 0 and
    // only feed estimates outside the ROI, which the NMS ignores
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<uint8_t*>(io.img(item)), (short)0, pitch * H, 0x00020000);
    auto load_row = [&](int yp) -> uint32_t {
        return __builtin_amdgcn_raw_buffer_load_b32(rs, yp * pitch + cx.xb, 0, 0);
    };

    RespState st;
    st.cbase = RAW_UNUSED;
    st.cfill = RAW_CHUNK;                       // no chunk yet: the first survivors reserve one
    const int nsteps = (cx.oy_end - cx.oy) + 6;
    const int nsup = (nsteps + SUP - 1) / SUP;
    uint32_t P[SUP];
#pragma unroll
    for (int u = 0; u < SUP; ++u) P[u] = load_row(cx.oy - 3 + u);
    uint32_t Q[SUP];
#pragma unroll
    for (int u = 0; u < SUP; ++u) Q[u] = load_row(cx.oy - 3 + SUP + u);
    // warm-up super-step: rows t = 0..5 (no NMS output yet)
    resp_step<0, false, false, false>(st, P[0], 0, cx);
    resp_step<1, false, false, false>(st, P[1], 1, cx);
    resp_step<2, true, false, false>(st, P[2], 2, cx);
    resp_step<3, true, false, false>(st, P[3], 3, cx);
    resp_step<4, true, true, false>(st, P[4], 4, cx);
    resp_step<5, true, true, false>(st, P[5], 5, cx);
    for (int sup = 1; sup < nsup; ++sup) {
        const int t0 = SUP * sup;
#pragma unroll
        for (int u = 0; u < SUP; ++u) P[u] = Q[u];
        if (sup + 1 < nsup) {
#pragma unroll
            for (int u = 0; u < SUP; ++u) Q[u] = load_row(cx.oy - 3 + t0 + SUP + u);
        }
        resp_step<0, true, true, true>(st, P[0], t0 + 0, cx);
        resp_step<1, true, true, true>(st, P[1], t0 + 1, cx);
        resp_step<2, true, true, true>(st, P[2], t0 + 2, cx);
        resp_step<3, true, true, true>(st, P[3], t0 + 3, cx);
        resp_step<4, true, true, true>(st, P[4], t0 + 4, cx);
        resp_step<5, true, true, true>(st, P[5], t0 + 5, cx);
    }
    if (st.cbase != RAW_UNUSED) mark_unused(cx.raw, st.cbase + st.cfill, st.cbase + RAW_CHUNK, cx.lane);
}

// Exact scores of the survivors; flagged ones get the exact NMS against their in-ROI neighbours.
template <class IO>
__global__ __launch_bounds__(256) void corner_keys_kernel(IO io, int W, int H, int pitch, int mx, int my, uint8_t* ws,
                                                          int64_t item_bytes)
{
    const int item = blockIdx.y;
    if (io.off(item)) return;
    CandHeader* hd = hdr_of(ws, item_bytes, item);
    const uint32_t nraw = hd->raw_count;
    const uint4* raw = raw_of(ws, item_bytes, item, W, H);
    uint64_t* keys = keys_of(ws, item_bytes, item);
    uint32_t* idx = idx_of(ws, item_bytes, item, W, H);
    const uint8_t* img = io.img(item);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int rx0 = mx, rx1 = W - mx, ry0 = my, ry1 = H - my;
    __shared__ uint32_t s_wcnt[4], s_base;
    __shared__ uint64_t s_wmax[4];
    uint64_t mx_bits = 0;
    for (uint32_t b0 = blockIdx.x * 256u; b0 < nraw; b0 += gridDim.x * 256u) {
        const uint32_t i = b0 + threadIdx.x;
        bool keep = false;
        uint64_t kb = 0;
        uint32_t ix = 0;
        const uint4 r = i < nraw ? raw[i] : make_uint4(0u, 0u, 0u, RAW_UNUSED);
        if (r.w != RAW_UNUSED) {
            ix = r.w & 0x7FFFFFFFu;
            const double key = exact_key((int32_t)r.x, (int32_t)r.y, (int32_t)r.z);
            keep = key > 0.0;
            if (keep && (r.w >> 31)) {
                const int x = (int)(ix % (uint32_t)W), y = (int)(ix / (uint32_t)W);
                for (int dy = -1; dy <= 1 && keep; ++dy)
                    for (int dx = -1; dx <= 1; ++dx) {
                        const int nx = x + dx, ny = y + dy;
                        if ((dx == 0 && dy == 0) || nx < rx0 || nx >= rx1 || ny < ry0 || ny >= ry1) continue;
                        int32_t A, B, C;
                        tensor_from_image(img, pitch, nx, ny, A, B, C);
                        if (exact_key(A, B, C) > key) { keep = false; break; }
                    }
            }
            kb = (uint64_t)__double_as_longlong(key);
        }
        // one atomic per workgroup and iteration places the workgroup's kept candidates
        const uint64_t bal = __ballot(keep);
        if (lane == 0) s_wcnt[wv] = (uint32_t)__popcll(bal);
        __syncthreads();
        if (threadIdx.x == 0) {
            const uint32_t tot = (s_wcnt[0] + s_wcnt[1]) + (s_wcnt[2] + s_wcnt[3]);
            s_base = tot ? atomicAdd(&hd->count, tot) : 0u;
        }
        __syncthreads();
        uint32_t pos = s_base;
        for (int w = 0; w < wv; ++w) pos += s_wcnt[w];
        pos += __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
        if (keep) {
            keys[pos] = kb;
            idx[pos] = ix;
            if (kb > mx_bits) mx_bits = kb;
        }
        __syncthreads();
    }
    // the largest kept key: one atomic per workgroup
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const uint64_t t = __shfl_xor(mx_bits, o, 64);
        mx_bits = t > mx_bits ? t : mx_bits;
    }
    if (lane == 0) s_wmax[wv] = mx_bits;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t m = s_wmax[0];
        for (int w = 1; w < 4; ++w) m = s_wmax[w] > m ? s_wmax[w] : m;
        if (m) atomicMax((unsigned long long*)&hd->lmax_bits, (unsigned long long)m);
    }
}

// composite key: larger is earlier in the selection order
__device__ __forceinline__ u128 comp(uint64_t kb, uint32_t ix, uint64_t base)
{
    return ((u128)(kb - base) << 32) | (u128)(0xFFFFFFFFu - ix);
}

__device__ __forceinline__ bool before(uint64_t ka, uint32_t ia, uint64_t kb, uint32_t ib)
{
    return ka > kb || (ka == kb && ia < ib);
}

// Calls f(key, index) for every candidate of the list, thread tid taking i = tid, tid + 1024, ...
// Eight loads per thread are issued before any is used, so a pass is not a chain of dependent
// global-memory latencies.
template <typename F>
__device__ __forceinline__ void for_each_key(const uint64_t* keys, const uint32_t* idx, uint32_t N, int tid, F f)
{
    constexpr int UNR = 8;
    for (uint32_t i0 = tid; i0 < N; i0 += 1024 * UNR) {
        uint64_t kb[UNR];
        uint32_t ix[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            const uint32_t i = i0 + 1024u * u;
            kb[u] = i < N ? keys[i] : 0;
            ix[u] = i < N ? idx[i] : 0;
        }
#pragma unroll
        for (int u = 0; u < UNR; ++u)
            if (i0 + 1024u * u < N) f(kb[u], ix[u]);
    }
}

template <class IO>
__global__ __launch_bounds__(1024) void corner_select_kernel(uint8_t* ws, int64_t item_bytes, int W, int H, IO io,
                                                             int Kmax, double quality, int min_dist, int capacity)
{
    const int item = blockIdx.x;
    if (io.off(item)) return;
    // per-item corner budget, clamped to [0, Kmax]
    const int K = io.budget(item, Kmax);
    float* __restrict__ xy_out = io.xy_of(item);
    double* __restrict__ score_out = io.score_of(item);
    __shared__ uint64_t bkey[CAP];
    __shared__ uint32_t bidx[CAP];
    __shared__ uint32_t hist[NBIN];
    __shared__ int32_t acc_x[VS_MAX_CORNERS];
    __shared__ int32_t acc_y[VS_MAX_CORNERS];
    __shared__ uint32_t s_conf[64];
    __shared__ __attribute__((aligned(16))) uint8_t s_mbits[64 * 16];
    __shared__ int32_t s_cx[64], s_cy[64];
    __shared__ int s_nacc, s_bcount, s_digit, s_done;
    __shared__ uint32_t s_need, s_above, s_sel_in_bin;

    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    CandHeader* hd = hdr_of(ws, item_bytes, item);
    const uint32_t N = hd->count;
    const uint64_t lmax_bits = hd->lmax_bits;
    const uint64_t* keys = keys_of(ws, item_bytes, item);
    const uint32_t* idx = idx_of(ws, item_bytes, item, W, H);
    const double lmax = __longlong_as_double((long long)lmax_bits);
    const double thr = __dmul_rn(quality, lmax);
    const uint64_t base = (uint64_t)__double_as_longlong(thr);
    const int64_t d2 = (int64_t)min_dist * min_dist;

    if (tid == 0) { s_nacc = 0; s_done = !(lmax > 0.0) || K <= 0; }
    __syncthreads();

    // keys requested per batch: the greedy typically consumes about 1.2 K candidates, so 1.5 K keeps
    // one batch (and a 2048-element sort for K up to ~1300) in the common case
    const uint32_t batch = (uint32_t)min(BATCH, max(512, K + K / 2));
    const uint64_t span = lmax_bits >= base ? lmax_bits - base : 0;
    const int nbits = (span ? 64 - __clzll((long long)span) : 0) + 32;
    bool unbounded = true;
    u128 U = 0;                    // exclusive upper bound on composite keys still to process

    while (!s_done) {
        // ---- 1) radix select the cut T: all eligible keys in [T, U) form the batch. The first digit
        // pass also counts the eligible keys: none left ends the selection, and when they all fit the
        // batch is all of them (T = 0).
        u128 T = 0;
        bool none_left = false;
        {
            int shift = nbits;
            u128 prefix = 0;
            if (tid == 0) { s_need = batch; s_above = 0; }
            __syncthreads();
            for (int pass = 0;; ++pass) {
                const int db = shift < DIGIT ? shift : DIGIT;
                const int pshift = shift;             // prefix covers bits >= pshift
                shift -= db;
                for (int b = tid; b < NBIN; b += 1024) hist[b] = 0;
                __syncthreads();
                for_each_key(keys, idx, N, tid, [&](uint64_t kb, uint32_t ix) {
                    bool in = kb >= base;
                    u128 v = 0;
                    if (in) {
                        v = comp(kb, ix, base);
                        in = (unbounded || v < U) && !(pshift < 128 && (v >> pshift) != prefix);
                    }
                    // most keys fall into a few low bins: the lanes sharing the first active lane's bin
                    // add in one atomic, the others one each
                    const uint32_t b = in ? ((uint32_t)(v >> shift) & ((1u << db) - 1u)) : 0xFFFFFFFFu;
                    const uint32_t b0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)b);
                    const uint64_t same = __ballot(in && b == b0);
                    if (same && lane == (int)__builtin_ctzll(same)) atomicAdd(&hist[b0], (uint32_t)__popcll(same));
                    if (in && b != b0) atomicAdd(&hist[b], 1u);
                });
                __syncthreads();
                // suffix sums from the top digit (Hillis-Steele in place over NBIN bins)
                for (int o = 1; o < NBIN; o <<= 1) {
                    uint32_t add[2] = {0, 0};
                    for (int q = 0; q < 2; ++q) {
                        const int b = tid + q * 1024;
                        if (b + o < NBIN) add[q] = hist[b + o];
                    }
                    __syncthreads();
                    for (int q = 0; q < 2; ++q) hist[tid + q * 1024] += add[q];
                    __syncthreads();
                }
                // hist[b] is now the count of keys with digit >= b; hist[0] counts every eligible key
                if (pass == 0 && hist[0] <= CAP) {
                    none_left = hist[0] == 0;
                    break;
                }
                const uint32_t need = s_need;
                if (tid == 0) { s_digit = 0; s_sel_in_bin = hist[0]; }
                __syncthreads();
                for (int q = 0; q < 2; ++q) {
                    const int b = tid + q * 1024;
                    if (b >= (1 << db)) continue;
                    const uint32_t ge = hist[b];
                    const uint32_t gt = (b + 1 < NBIN) ? hist[b + 1] : 0;
                    if (gt < need && ge >= need) { s_digit = b; s_sel_in_bin = ge - gt; }
                }
                __syncthreads();
                const int dstar = s_digit < 0 ? 0 : (s_digit >= NBIN ? NBIN - 1 : s_digit);
                const uint32_t gt_star = (dstar + 1 < NBIN) ? hist[dstar + 1] : 0;
                const uint32_t in_bin = s_sel_in_bin;
                const uint32_t above_prev = s_above;
                __syncthreads();
                prefix = (prefix << db) | (u128)(uint32_t)dstar;
                const uint32_t above = above_prev + gt_star;
                if (above + in_bin <= CAP || shift == 0) {
                    T = prefix << shift;
                    break;
                }
                if (tid == 0) { s_above = above; s_need = need - gt_star; }
                __syncthreads();
            }
        }
        if (none_left) break;

        // ---- 2) gather [T, U) into LDS
        if (tid == 0) s_bcount = 0;
        __syncthreads();
        for_each_key(keys, idx, N, tid, [&](uint64_t kb, uint32_t ix) {
            bool take = kb >= base;
            if (take) {
                const u128 v = comp(kb, ix, base);
                take = !(v < T || (!unbounded && v >= U));
            }
            // one atomic per wave for the wave's selected keys
            const uint64_t m = __ballot(take);
            if (!m) return;
            int first = 0;
            if (lane == (int)__builtin_ctzll(m)) first = atomicAdd(&s_bcount, __popcll(m));
            first = __shfl(first, (int)__builtin_ctzll(m), 64);
            const int slot = first + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
            if (take && slot < CAP) {  // always true by construction of T; keeps LDS writes in range
                bkey[slot] = kb;
                bidx[slot] = ix;
            }
        });
        __syncthreads();
        const int bc = s_bcount < CAP ? s_bcount : CAP;
        int p2 = 1;
        while (p2 < bc) p2 <<= 1;
        for (int i = bc + tid; i < p2; i += 1024) { bkey[i] = 0; bidx[i] = 0xFFFFFFFFu; }
        __syncthreads();

        // ---- 3) bitonic sort, earliest first
        for (int k = 2; k <= p2; k <<= 1) {
            for (int j = k >> 1; j > 0; j >>= 1) {
                for (int i = tid; i < p2; i += 1024) {
                    const int l = i ^ j;
                    if (l > i) {
                        const bool up = (i & k) == 0;
                        const uint64_t ka = bkey[i], kb2 = bkey[l];
                        const uint32_t ia = bidx[i], ib = bidx[l];
                        const bool swap = up ? before(kb2, ib, ka, ia) : before(ka, ia, kb2, ib);
                        if (swap) { bkey[i] = kb2; bkey[l] = ka; bidx[i] = ib; bidx[l] = ia; }
                    }
                }
                __syncthreads();
            }
        }

        // ---- 4) greedy acceptance, 64 candidates at a time. Wave 0 stages a group's coordinates. All
        // waves then test the group against the corners accepted so far and fill the group's 64 x 64
        // matrix of too-close earlier members. Wave 0 accepts the members clear of both at once and
        // walks only the contested ones in order; then it stages the next group. Two barriers a group.
        if (tid < 64) {
            s_conf[tid] = 0;
            if (tid < bc) {
                const uint32_t ix = bidx[tid];
                s_cx[tid] = (int32_t)(ix % (uint32_t)W);
                s_cy[tid] = (int32_t)(ix / (uint32_t)W);
            }
        }
        __syncthreads();
        for (int g0 = 0; g0 < bc; g0 += 64) {
            const int na = s_nacc;
            if (na >= K) break;
            const int gn = min(64, bc - g0);                  // members in this group
            if (lane < gn) {
                const int cx = s_cx[lane], cy = s_cy[lane];
                bool conf = false;
                // wave wv checks accepted corners wv, wv + 16, ...; four independent reads per step
                for (int j = wv; j < na && !conf; j += 64) {
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int jj = j + 16 * u;
                        if (jj < na) {
                            const int64_t dx = cx - acc_x[jj], dy = cy - acc_y[jj];
                            conf = conf || dx * dx + dy * dy < d2;
                        }
                    }
                }
                if (conf) s_conf[lane] = 1;
                // members 4 wv .. 4 wv + 3 of the group that come before this lane and are too close
                uint32_t bits = 0;
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const int j = 4 * wv + b;
                    if (j < lane) {
                        const int64_t dx = cx - s_cx[j], dy = cy - s_cy[j];
                        if (dx * dx + dy * dy < d2) bits |= 1u << b;
                    }
                }
                s_mbits[lane * 16 + wv] = (uint8_t)bits;
            } else {
                s_mbits[lane * 16 + wv] = 0;
            }
            __syncthreads();
            if (wv == 0) {
                const bool valid = lane < gn;
                const int cx = valid ? s_cx[lane] : 0, cy = valid ? s_cy[lane] : 0;
                const bool pre_ok = valid && s_conf[lane] == 0;
                const uint64_t ok = __ballot(pre_ok);
                const uint4 mb = *reinterpret_cast<const uint4*>(&s_mbits[lane * 16]);
                const uint32_t w4[4] = {mb.x, mb.y, mb.z, mb.w};
                uint64_t mask = 0;
#pragma unroll
                for (int q = 0; q < 16; ++q) mask |= (uint64_t)((w4[q >> 2] >> (8 * (q & 3))) & 0xFu) << (4 * q);
                mask &= ok;                                   // earlier members still eligible and too close
                uint64_t acc = __ballot(pre_ok && mask == 0); // no earlier eligible member too close
                uint64_t contested = ok & ~acc;
                while (contested) {
                    const int k = __builtin_ctzll(contested);
                    contested &= contested - 1;
                    const uint32_t mlo = __builtin_amdgcn_readlane((uint32_t)mask, k);
                    const uint32_t mhi = __builtin_amdgcn_readlane((uint32_t)(mask >> 32), k);
                    if (!((((uint64_t)mhi << 32) | mlo) & acc)) acc |= 1ull << k;
                }
                // the corner budget keeps the first K - na acceptances in group order
                const int allowed = K - na;
                const int rank_in = __popcll(acc & ((1ull << lane) - 1ull));
                if (((acc >> lane) & 1ull) && rank_in < allowed) {
                    const int rank = na + rank_in;
                    acc_x[rank] = cx;
                    acc_y[rank] = cy;
                    float* o = xy_out + rank * 2;
                    o[0] = (float)cx;
                    o[1] = (float)cy;
                    if (score_out) score_out[rank] = __longlong_as_double((long long)bkey[g0 + lane]);
                }
                if (lane == 0) s_nacc = na + min(__popcll(acc), allowed);
                // stage the next group
                s_conf[lane] = 0;
                if (g0 + 64 + lane < bc) {
                    const uint32_t ix = bidx[g0 + 64 + lane];
                    s_cx[lane] = (int32_t)(ix % (uint32_t)W);
                    s_cy[lane] = (int32_t)(ix / (uint32_t)W);
                }
            }
            __syncthreads();
        }
        if (tid == 0) {
            if (s_nacc >= K || T == 0) s_done = 1;
        }
        U = T;
        unbounded = false;
        __syncthreads();
    }
    __syncthreads();
    const int na = s_nacc;
    uint8_t* alive_out = io.alive_of(item);
    for (int k = tid; k < capacity; k += 1024) alive_out[k] = k < na ? 1 : 0;
    if (tid == 0) *io.count_of(item) = na;
}

// the four detection launches over n items
template <class IO>
int launch_detect(const IO& io, int n, int width, int height, int pitch, const vs_detect_params& p, int Kmax,
                  int capacity, uint8_t* w8, hipStream_t s)
{
    const int64_t ib = per_item_bytes(width, height);
    detect_init_kernel<<<(n + 255) / 256, 256, 0, s>>>(w8, ib, n, io);
    int e = vs::check_launch("vs_detect_corners(init)");
    if (e) return e;
    const int rw = width - 2 * p.roi_mx, rh = height - 2 * p.roi_my;
    // each output row belongs to one wave's segment and the survivors are sorted afterwards, so the
    // segment height only trades per-wave warm-up rows against waves per frame
    const int sr = vs::detect_segment_rows(n, SR_FEW, SR);   // >= SR_FEW, which sizes the survivor list
    const int strips = (rw + SW - 1) / SW, segs = (rh + sr - 1) / sr;
    const int64_t nwaves = (int64_t)n * strips * segs;
    corner_response_kernel<<<(unsigned)((nwaves + 3) / 4), 256, 0, s>>>(io, width, height, pitch, p.roi_mx, p.roi_my, n,
                                                                      strips, segs, sr, w8, ib);
    e = vs::check_launch("vs_detect_corners(response)");
    if (e) return e;
    // survivors are a small fraction of the ROI: 32 blocks per item stride over them (256 for
    // batches of at most 8 frames)
    corner_keys_kernel<<<dim3(n <= 8 ? 256 : 32, n), 256, 0, s>>>(io, width, height, pitch, p.roi_mx, p.roi_my, w8, ib);
    e = vs::check_launch("vs_detect_corners(keys)");
    if (e) return e;
    corner_select_kernel<<<n, 1024, 0, s>>>(w8, ib, width, height, io, Kmax, p.quality, p.min_dist, capacity);
    return vs::check_launch("vs_detect_corners(select)");
}

int check_detect(const vs_detect_params& p, int width, int height, int pitch, int capacity)
{
    if (width < 8 || height < 8 || pitch < width) return vs::set_error(VS_ERR_INVALID, "vs_detect_corners: bad size");
    if (capacity > VS_MAX_CORNERS) return vs::set_error(VS_ERR_UNSUPPORTED, "vs_detect_corners: capacity > %d", VS_MAX_CORNERS);
    if (p.max_corners < 0 || p.max_corners > capacity || capacity <= 0)
        return vs::set_error(VS_ERR_INVALID, "vs_detect_corners: need 0 <= max_corners <= capacity");
    if (p.roi_mx < 2 || p.roi_my < 2 || width - 2 * p.roi_mx <= 0 || height - 2 * p.roi_my <= 0)
        return vs::set_error(VS_ERR_INVALID, "vs_detect_corners: ROI margins must be >= 2 and leave a non-empty ROI");
    if (p.min_dist < 0 || !(p.quality >= 0.0) || p.quality > 1.0)
        return vs::set_error(VS_ERR_INVALID, "vs_detect_corners: bad min_dist or quality");
    if ((int64_t)pitch * height >= (int64_t)1 << 31)
        return vs::set_error(VS_ERR_UNSUPPORTED, "vs_detect_corners: frame too large");
    return VS_OK;
}

}  // namespace

extern "C" size_t vs_detect_workspace(int32_t width, int32_t height, int32_t n)
{
    if (width <= 0 || height <= 0 || n <= 0) return 0;
    return (size_t)per_item_bytes(width, height) * (size_t)n;
}

extern "C" int vs_detect_corners(const uint8_t* frames, int64_t frame_stride, int32_t width, int32_t height,
                                 int32_t pitch, int32_t n, int32_t istride, const int32_t* gate, int32_t gate_min,
                                 const vs_detect_params* p, int32_t capacity, float* xy, double* score,
                                 int32_t* count, uint8_t* alive, void* workspace, size_t ws_bytes, void* stream)
{
    if (!p || (n > 0 && (!frames || !xy || !count || !alive || !workspace)))
        return vs::set_error(VS_ERR_INVALID, "vs_detect_corners: null argument");
    if (n < 0 || istride < 1) return vs::set_error(VS_ERR_INVALID, "vs_detect_corners: bad size");
    int e = check_detect(*p, width, height, pitch, capacity);
    if (e) return e;
    if (n == 0) return VS_OK;
    if (n > 65535) return vs::set_error(VS_ERR_INVALID, "vs_detect_corners: more than 65535 items");
    if (n > 1 && frame_stride < (int64_t)pitch * height)
        return vs::set_error(VS_ERR_INVALID, "vs_detect_corners: frame stride overlaps items");
    const size_t need = vs_detect_workspace(width, height, n);
    if (ws_bytes < need) return vs::set_error(VS_ERR_WORKSPACE, "vs_detect_corners: workspace %zu < %zu", ws_bytes, need);
    if (reinterpret_cast<uintptr_t>(workspace) & 255)
        return vs::set_error(VS_ERR_INVALID, "vs_detect_corners: workspace must be 256-byte aligned");
    const Strided io{frames, frame_stride, istride, gate, gate_min, p->max_corners_per_item, capacity, xy, score, count,
                     alive};
    return launch_detect(io, n, width, height, pitch, *p, p->max_corners, capacity, static_cast<uint8_t*>(workspace),
                         vs::as_stream(stream));
}

namespace vs {

// the detection of every item of a batched step (items whose detection is not due return at once);
// the workspace holds vs_detect_workspace(W, H, n) bytes
int step_detect(const StepView& v, int n, int W, int H, const vs_detect_params& p, uint8_t* ws, hipStream_t s)
{
    if (n <= 0) return VS_OK;
    vs_detect_params q = p;
    q.max_corners = v.capacity;   // each stream's own budget applies (clamped to the capacity)
    const int e = check_detect(q, W, H, W, v.capacity);
    if (e) return e;
    return launch_detect(Step{v}, n, W, H, W, q, v.capacity, v.capacity, ws, s);
}

}  // namespace vs
