// detect_corners: Shi-Tomasi response + 3x3 NMS over the ROI, then the ordered greedy top-K.
//
// Kernel 1 (corner_response): each wave walks down a 240-column strip of the ROI, 60 output rows at a
// time; lane i owns 4 columns. Per pixel row it forms, in registers, the Sobel terms, the tensor
// products and their 3x3 box sums (all integers below 2^24, so exact in FP32), an FP32 estimate of
// the score with a bounded relative error, and a separable 3x3 max of the estimates; neighbouring
// lanes' edge columns arrive by DPP wave shifts. A pixel whose neighbours' estimates are all below
// its own by more than the error band survives; one whose neighbours are above by more than the band
// is dropped; a pixel inside the band survives flagged. Survivors queue in the wave's LDS as their
// exact box-summed tensor (A, B, C) and pixel index. Every 64 queued survivors, one per lane, get
// their exact binary64 score 2 det / (tr + sqrt(disc)); a flagged one is compared exactly against its
// in-ROI neighbours, recomputed from the image. The survivors that remain queue again in LDS as
// (score bits, index) and are appended to the item's candidate lists 256 at a time with one atomic;
// the wave's largest score is folded into the item's maximum with one integer atomic max on the
// score's bit pattern (non-negative doubles order like their bits). The candidates are exactly the
// set of 3x3 maxima of the exact scores; nothing but them reaches global memory.
//
// Kernel 2 (corner_select): one 1024-thread workgroup per item. Candidates below
// quality * max are dropped. The order is (score desc, y asc, x asc), i.e. the composite key
// V = (bits(score) - bits(threshold)) * 2^32 + (2^32 - 1 - y * W - x) taken descending. Batches of
// the next ~2048 keys are cut out by a most-significant-digit radix select (11-bit digits; the
// passes over the score bits read only the scores), bitonic-sorted in LDS and fed to the greedy
// minimum-distance test 64 at a time: all 16 waves test a group against the accepted set, then one
// wave resolves conflicts inside the group in order. The result equals the sequential greedy over
// the full sorted list.
#include "vs_common.hpp"

namespace {

typedef unsigned __int128 u128;

struct CandHeader {
    uint32_t count;        // candidates (exact 3x3 maxima) in the key/index lists
    uint32_t unused;
    uint64_t lmax_bits;    // bit pattern of the largest candidate score (0: none yet)
};

// Score histogram of an item's candidates: bin b counts the scores whose bits, shifted right by 48
// (exponent and 4 leading mantissa bits: 1/16 octave), equal b + BIN_BASE, clamped to [0, NBIN_S);
// bin 0 holds everything below 2^-25 and the last everything from 2^25 on (the exact scores of
// 8-bit images lie between 2^-25 and 2^25). Monotone in the score.
constexpr int BIN_SHIFT = 48;
constexpr int NBIN_S = 50 * 16;
constexpr int64_t BIN_BASE = (int64_t)(1023 - 25) * 16;
__host__ __device__ inline int score_bin(uint64_t kb)
{
    const int64_t b = (int64_t)(kb >> BIN_SHIFT) - BIN_BASE;
    return b < 0 ? 0 : (b >= NBIN_S ? NBIN_S - 1 : (int)b);
}
// the smallest score bits of bin b (1 <= b < NBIN_S): score_bin(k) >= b exactly when k >= bin_low(b)
__host__ __device__ inline uint64_t bin_low(int b) { return (uint64_t)(b + BIN_BASE) << BIN_SHIFT; }

constexpr int64_t HIST = 256;                       // the histogram follows the 256-byte header
constexpr int64_t HDR = HIST + ((4 * NBIN_S + 255) & ~255);
constexpr int SW = 240;         // output columns per wave strip (lanes 1..62 of 64 x 4 columns)
constexpr int SUP = 6;          // rows per unrolled super-step (period of the register rotation)
constexpr int SR = 60;          // output rows per wave: the pipeline runs SR + 6 pixel rows
constexpr int SR_FEW = 12;      // rows per wave for batches of at most 8 frames (more waves per frame)
constexpr int CAP = 4096;       // LDS batch capacity of the selection
constexpr int BATCH = 2048;     // keys requested per batch
constexpr int DIGIT = 11;
constexpr int NBIN = 1 << DIGIT;
// LDS queues of one response wave. Survivors are scored 64 at a time, so fewer than 64 wait after a
// row's scoring and one row adds at most 4 x 62; kept candidates are appended KFLUSH at a time, so
// fewer than KFLUSH wait before a chunk adds at most 64.
constexpr int QCAP = 320;
constexpr int KFLUSH = 256;
constexpr int KCAP = KFLUSH + 64;
static_assert(63 + 4 * 62 <= QCAP && KFLUSH - 1 + 64 <= KCAP, "queue capacities");

struct WaveQueues {
    uint4 surv[QCAP];        // A, B, C (bits of exact floats), pixel index | flag << 31
    uint64_t key[KCAP];      // bits of the exact score
    uint32_t idx[KCAP];
    uint32_t hist[NBIN_S];   // the wave's score histogram of its kept candidates
};
constexpr int RESP_WAVES = 4;   // waves per response workgroup

// per item: header | score histogram | keys (8 B each) | indices (4 B), each list with room for one
// entry per pixel
__host__ __device__ inline int64_t per_item_bytes(int w, int h)
{
    const int64_t c = (int64_t)w * h;
    return (HDR + 12 * c + 255) & ~(int64_t)255;
}

__device__ __forceinline__ CandHeader* hdr_of(uint8_t* ws, int64_t item_bytes, int item)
{
    return reinterpret_cast<CandHeader*>(ws + item * item_bytes);
}
__device__ __forceinline__ uint32_t* hist_of(uint8_t* ws, int64_t item_bytes, int item)
{
    return reinterpret_cast<uint32_t*>(ws + item * item_bytes + HIST);
}
__device__ __forceinline__ uint64_t* keys_of(uint8_t* ws, int64_t item_bytes, int item)
{
    return reinterpret_cast<uint64_t*>(ws + item * item_bytes + HDR);
}
__device__ __forceinline__ uint32_t* idx_of(uint8_t* ws, int64_t item_bytes, int item, int w, int h)
{
    return reinterpret_cast<uint32_t*>(ws + item * item_bytes + HDR + 8 * (int64_t)w * h);
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
    const int i = blockIdx.x;   // one workgroup per item
    if (i >= n || io.off(i)) return;
    if (threadIdx.x == 0) {
        CandHeader* h = hdr_of(ws, item_bytes, i);
        h->count = 0;
        h->lmax_bits = 0;
    }
    uint32_t* hist = hist_of(ws, item_bytes, i);
    for (int b = threadIdx.x; b < NBIN_S; b += blockDim.x) hist[b] = 0;
}


// Exact binary64 score 2 det / (tr + sqrt(disc)) of the box-summed tensor (integers, passed as
// doubles). With |A|, |B|, |C| < 2^24 every product and sum below is an integer below 2^53, so det,
// tr and disc are exact and equal to their 64-bit integer values; sqrt, add and divide are single
// correctly rounded operations.
__device__ __forceinline__ double exact_key(double a, double b, double c)
{
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
__device__ __forceinline__ float approx_key(float a, float b, float c)
{
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
// side maxima). All indices are compile-time constants after unrolling. Every tensor value is an
// integer below 2^24 in magnitude held exactly in FP32.
struct RespState {
    float dx[3][4], sy[3][4];
    float ha[3][4], hb[3][4], hc[3][4];
    float sa[2][4], sb[2][4], sc[2][4];
    float sv[2][4], hm[3][4], sd[2][4];
    int qn, kn;          // queued survivors and queued kept candidates (wave-uniform)
    uint64_t kmax;       // the lane's largest kept score bits
};

struct RespCtx {
    int lane, xb, oy, oy_end;
    int rx0, rx1, ry0, ry1;
    int out_lo, out_hi;          // output columns of this strip
    int W, pitch;
    const uint8_t* img;
    uint32_t* count;             // the item's candidate count
    uint32_t* hist;              // the item's score histogram
    uint64_t* keys;              // the item's candidate lists (room for one entry per pixel)
    uint32_t* idx;
    WaveQueues* q;               // this wave's LDS queues
};

// Appends the queued kept candidates to the item's lists (one atomic) and empties the queue.
__device__ __forceinline__ void flush_kept(RespState& st, const RespCtx& cx)
{
    vs::wave_lds_sync();
    uint32_t b = 0;
    if (cx.lane == 0) b = atomicAdd(cx.count, (uint32_t)st.kn);
    const uint32_t base = (uint32_t)__builtin_amdgcn_readfirstlane((int)b);
    for (int i = cx.lane; i < st.kn; i += 64) {
        cx.keys[base + i] = cx.q->key[i];
        cx.idx[base + i] = cx.q->idx[i];
    }
    st.kn = 0;
    vs::wave_lds_sync();
}

// whether an in-ROI neighbour of (x, y) has an exact score above `key` (the exact NMS of a flagged
// survivor; the neighbours' tensors are recomputed from the image)
__device__ bool beaten_by_neighbour(const RespCtx& cx, int x, int y, double key)
{
    for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
            const int nx = x + dx, ny = y + dy;
            if ((dx == 0 && dy == 0) || nx < cx.rx0 || nx >= cx.rx1 || ny < cx.ry0 || ny >= cx.ry1) continue;
            int32_t A, B, C;
            tensor_from_image(cx.img, cx.pitch, nx, ny, A, B, C);
            if (exact_key((double)A, (double)B, (double)C) > key) return true;
        }
    return false;
}

// Exact scores of the queued survivors [h, h + cnt), cnt <= 64, one per lane; those that remain
// queue as kept candidates, written out once KFLUSH are queued.
__device__ __forceinline__ void score_chunk(RespState& st, const RespCtx& cx, int h, int cnt)
{
    vs::wave_lds_sync();
    bool keep = false;
    uint64_t kb = 0;
    uint32_t ix = 0;
    if (cx.lane < cnt) {
        const uint4 r = cx.q->surv[h + cx.lane];
        ix = r.w & 0x7FFFFFFFu;
        const double key = exact_key((double)__uint_as_float(r.x), (double)__uint_as_float(r.y),
                                     (double)__uint_as_float(r.z));
        keep = key > 0.0;
        if (keep && (r.w >> 31))
            keep = !beaten_by_neighbour(cx, (int)(ix % (uint32_t)cx.W), (int)(ix / (uint32_t)cx.W), key);
        kb = (uint64_t)__double_as_longlong(key);
    }
    const uint64_t bal = __ballot(keep);
    if (keep) {
        const int pos = st.kn + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
        cx.q->key[pos] = kb;
        cx.q->idx[pos] = ix;
        atomicAdd(&cx.q->hist[score_bin(kb)], 1u);
        if (kb > st.kmax) st.kmax = kb;
    }
    st.kn += __popcll(bal);
    if (st.kn >= KFLUSH) flush_kept(st, cx);
}

// One pixel-row step. T is the step number modulo SUP; GRAD/BOX/NMS switch the pipeline stages on.
// Pixel row yp = oy - 3 + t; gradients for row yp - 1; box sums and estimates for row yp - 2; NMS
// decisions for row yp - 3.
template <int T, bool GRAD, bool BOX, bool NMS>
__device__ __forceinline__ void resp_step(RespState& st, uint32_t P, int t, const RespCtx& cx)
{
    constexpr int i3 = T % 3, m3 = (T + 2) % 3, mm3 = (T + 1) % 3;   // t, t-1, t-2 (mod 3)
    constexpr int i2 = T % 2, m2 = (T + 1) % 2;                       // t, t-1 (mod 2)
    const uint32_t L = (uint32_t)dpp_i<DPP_SHR>((int)P), R = (uint32_t)dpp_i<DPP_SHL>((int)P);
    const float p0 = (float)(P & 0xffu), p1 = (float)((P >> 8) & 0xffu), p2 = (float)((P >> 16) & 0xffu);
    const float p3 = (float)(P >> 24), pl = (float)(L >> 24), pr = (float)(R & 0xffu);
    // horizontal Sobel terms: (1,2,1) smoothing and central difference
    st.sy[i3][0] = fmaf(2.0f, p0, pl) + p1;
    st.sy[i3][1] = fmaf(2.0f, p1, p0) + p2;
    st.sy[i3][2] = fmaf(2.0f, p2, p1) + p3;
    st.sy[i3][3] = fmaf(2.0f, p3, p2) + pr;
    st.dx[i3][0] = p1 - pl;
    st.dx[i3][1] = p2 - p0;
    st.dx[i3][2] = p3 - p1;
    st.dx[i3][3] = pr - p2;
    if constexpr (GRAD) {
        float A[4], B[4], C[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const float gx = fmaf(2.0f, st.dx[m3][c], st.dx[mm3][c]) + st.dx[i3][c];
            const float gy = st.sy[i3][c] - st.sy[mm3][c];
            A[c] = gx * gx;
            B[c] = gx * gy;
            C[c] = gy * gy;
        }
        const float al = dpp_f<DPP_SHR>(A[3]), ar = dpp_f<DPP_SHL>(A[0]);
        const float bl = dpp_f<DPP_SHR>(B[3]), br = dpp_f<DPP_SHL>(B[0]);
        const float cl = dpp_f<DPP_SHR>(C[3]), cr = dpp_f<DPP_SHL>(C[0]);
        // 3-column sums; the middle pair is shared by columns 1 and 2 (integers: any order is exact)
        const float a12 = A[1] + A[2], b12 = B[1] + B[2], c12 = C[1] + C[2];
        st.ha[i3][0] = (al + A[0]) + A[1];
        st.hb[i3][0] = (bl + B[0]) + B[1];
        st.hc[i3][0] = (cl + C[0]) + C[1];
        st.ha[i3][1] = A[0] + a12;
        st.hb[i3][1] = B[0] + b12;
        st.hc[i3][1] = C[0] + c12;
        st.ha[i3][2] = a12 + A[3];
        st.hb[i3][2] = b12 + B[3];
        st.hc[i3][2] = c12 + C[3];
        st.ha[i3][3] = (A[2] + A[3]) + ar;
        st.hb[i3][3] = (B[2] + B[3]) + br;
        st.hc[i3][3] = (C[2] + C[3]) + cr;
    }
    if constexpr (BOX) {
        const int yb = cx.oy - 5 + t;
        const bool row_in = yb >= cx.ry0 && yb < cx.ry1;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            st.sa[i2][c] = (st.ha[mm3][c] + st.ha[m3][c]) + st.ha[i3][c];
            st.sb[i2][c] = (st.hb[mm3][c] + st.hb[m3][c]) + st.hb[i3][c];
            st.sc[i2][c] = (st.hc[mm3][c] + st.hc[m3][c]) + st.hc[i3][c];
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
        int tot = 0;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            bal[c] = __ballot(surv[c]);
            tot += __popcll(bal[c]);
        }
        if (tot) {
            // queue the row's survivors behind the waiting ones (fewer than 64 wait: capacity QCAP)
            int base = st.qn;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const uint32_t lo = (uint32_t)bal[c], hi = (uint32_t)(bal[c] >> 32);
                const int pos = base + (int)__builtin_amdgcn_mbcnt_hi(hi, __builtin_amdgcn_mbcnt_lo(lo, 0u));
                if (surv[c]) {
                    const uint32_t ix = (uint32_t)(yn * cx.W + cx.xb + c) | (flag[c] ? 0x80000000u : 0u);
                    cx.q->surv[pos] = make_uint4(__float_as_uint(st.sa[m2][c]), __float_as_uint(st.sb[m2][c]),
                                                 __float_as_uint(st.sc[m2][c]), ix);
                }
                base += __popcll(bal[c]);
            }
            st.qn = base;
            if (st.qn >= 64) {
                int h = 0;
                do {
                    score_chunk(st, cx, h, 64);
                    h += 64;
                } while (st.qn - h >= 64);
                // move the rest (fewer than 64 entries, disjoint from their new place as h >= 64) to the front
                const int rest = st.qn - h;
                vs::wave_lds_sync();
                if (cx.lane < rest) cx.q->surv[cx.lane] = cx.q->surv[h + cx.lane];
                vs::wave_lds_sync();
                st.qn = rest;
            }
        }
    }
}

template <class IO>
__global__ __launch_bounds__(64 * RESP_WAVES) __attribute__((amdgpu_waves_per_eu(3))) void corner_response_kernel(IO io, int W, int H, int pitch, int mx, int my,
                                                                          int n_items, int strips, int segs, int sr,
                                                                          uint8_t* ws, int64_t item_bytes)
{
    __shared__ WaveQueues s_q[RESP_WAVES];
    // one independent wave per (item, strip, segment); the wave index is read as a scalar, so the item,
    // its image and the buffer descriptor are known to be uniform (no per-load waterfall loops)
    const int gw = blockIdx.x * RESP_WAVES + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int per_item = strips * segs;
    const int item = gw / per_item;
    if (item >= n_items) return;
    if (io.off(item)) return;
    const int rem = gw - item * per_item;
    const int seg = rem / strips, strip = rem - seg * strips;

    RespCtx cx;
    cx.lane = threadIdx.x & 63;
    cx.W = W;
    cx.pitch = pitch;
    cx.rx0 = mx; cx.rx1 = W - mx; cx.ry0 = my; cx.ry1 = H - my;
    cx.out_lo = mx + SW * strip;
    cx.out_hi = min(cx.out_lo + SW, cx.rx1);
    cx.xb = ((cx.out_lo - 4) & ~3) + 4 * cx.lane;   // lanes 1..62 cover [out_lo, out_lo + SW)
    cx.oy = my + sr * seg;
    cx.oy_end = min(cx.oy + sr, cx.ry1);
    cx.img = vs::uniform_ptr(io.img(item));   // a batched step reads it from memory
    CandHeader* hd = hdr_of(ws, item_bytes, item);
    cx.count = &hd->count;
    cx.hist = hist_of(ws, item_bytes, item);
    cx.keys = keys_of(ws, item_bytes, item);
    cx.idx = idx_of(ws, item_bytes, item, W, H);
    cx.q = &s_q[threadIdx.x >> 6];

    // pixel rows are read through a buffer descriptor: rows or columns past the image read as 0 and
    // only feed estimates outside the ROI, which the NMS ignores
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t*>(cx.img), (short)0,
                                                                        pitch * H, 0x00020000);
    auto load_row = [&](int yp) -> uint32_t {
        return __builtin_amdgcn_raw_buffer_load_b32(rs, yp * pitch + cx.xb, 0, 0);
    };

    RespState st;
    st.qn = 0;
    st.kn = 0;
    st.kmax = 0;
    static_assert(NBIN_S % 4 == 0, "the histogram is cleared 16 bytes at a time");
    for (int b = 4 * cx.lane; b < NBIN_S; b += 4 * 64)   // ordered before use by the scoring's sync
        *reinterpret_cast<uint4*>(&cx.q->hist[b]) = make_uint4(0u, 0u, 0u, 0u);
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
    // the last survivors and kept candidates, then the wave's largest score (one atomic per wave)
    if (st.qn > 0) score_chunk(st, cx, 0, st.qn);
    if (st.kn > 0) flush_kept(st, cx);
    // the wave's histogram into the item's (one atomic per non-empty bin)
    vs::wave_lds_sync();
    for (int b = cx.lane; b < NBIN_S; b += 64) {
        const uint32_t h = cx.q->hist[b];
        if (h) atomicAdd(&cx.hist[b], h);
    }
    uint64_t m = st.kmax;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const uint64_t t = __shfl_xor(m, o, 64);
        m = t > m ? t : m;
    }
    if (cx.lane == 0 && m) atomicMax((unsigned long long*)&hd->lmax_bits, (unsigned long long)m);
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

// Whether two corners are closer than the minimum distance (d2 = its square). For frames whose
// sides are at most 32768 (D24) every coordinate difference fits 24-bit multiplies and the sum of
// squares stays below 2^31, so 32-bit arithmetic decides it exactly (d2 clamped to 2^32 - 1 leaves
// every decision unchanged); larger frames use 64-bit arithmetic.
template <bool D24>
__device__ __forceinline__ bool too_close(int ax, int ay, int bx, int by, uint32_t d2_32, int64_t d2)
{
    if constexpr (D24) {
        const int dx = ax - bx, dy = ay - by;
        return (uint32_t)__mul24(dy, dy) + (uint32_t)__mul24(dx, dx) < d2_32;
    } else {
        const int64_t dx = ax - bx, dy = ay - by;
        return dx * dx + dy * dy < d2;
    }
}
constexpr int D24_MAX_SIDE = 32768;

// One greedy group, first phase (every wave): member `lane` of the group at g0 (if lane < gn) is
// tested against the na accepted corners -- wave wv takes corners 4 wv .. 4 wv + 3, then 128 further
// on, ..., with two 16-byte reads of the same addresses by every lane per 4 corners -- and against
// the group's members 4 wv .. 4 wv + 3 that come before it. A conflict with an accepted corner sets
// s_conf[lane]; too-close earlier members set their bits in s_mask[lane].
template <bool D24>
__device__ __forceinline__ void greedy_test(const int2* bxy, const int2* acc_xy, int g0, int gn, int na, int lane,
                                            int wv, uint32_t d2_32, int64_t d2, uint32_t* s_conf, uint64_t* s_mask)
{
    if (lane >= gn) return;
    const int2 c = bxy[g0 + lane];
    bool conf = false;
    for (int j = 4 * wv; j < na && !conf; j += 2 * 64) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int jb = j + 64 * u;
            const int4 q0 = *reinterpret_cast<const int4*>(&acc_xy[jb]);
            const int4 q1 = *reinterpret_cast<const int4*>(&acc_xy[jb + 2]);
            const int qx[4] = {q0.x, q0.z, q1.x, q1.z}, qy[4] = {q0.y, q0.w, q1.y, q1.w};
            // every test is evaluated (bitwise, not short-circuit), so no branch splits the reads
#pragma unroll
            for (int v = 0; v < 4; ++v) conf |= (jb + v < na) & too_close<D24>(c.x, c.y, qx[v], qy[v], d2_32, d2);
        }
    }
    if (conf) s_conf[lane] = 1;
    uint64_t bits = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const int j = 4 * wv + b;
        const int2 o = bxy[g0 + j];        // j < 64 <= CAP - g0: inside the batch array
        bits |= (uint64_t)((j < lane) & too_close<D24>(c.x, c.y, o.x, o.y, d2_32, d2)) << j;
    }
    if (bits) atomicOr((unsigned long long*)&s_mask[lane], (unsigned long long)bits);
}

// Sorts the batch bkey/bidx[0, 1024 R) earliest first (bitonic network). Thread t holds elements
// w 64 R + h 64 + l (wave w, lane l, h < R) in registers: compare-exchanges with partners in the same
// lane or across lanes of the wave run in registers (the latter by shuffles); only the strides
// reaching another wave go through LDS, with two barriers each. Called by all 1024 threads.
template <int R>
__device__ void sort_batch(uint64_t* bkey, uint32_t* bidx, int tid)
{
    constexpr int S = 1024 * R;
    const int lane = tid & 63, wv = tid >> 6;
    uint64_t k[R];
    uint32_t x[R];
#pragma unroll
    for (int h = 0; h < R; ++h) {
        k[h] = bkey[wv * 64 * R + h * 64 + lane];
        x[h] = bidx[wv * 64 * R + h * 64 + lane];
    }
    for (int kk = 2; kk <= S; kk <<= 1) {
        for (int j = kk >> 1; j > 0; j >>= 1) {
            if (j >= 64 * R) {
                // partner in another wave
                __syncthreads();
#pragma unroll
                for (int h = 0; h < R; ++h) {
                    bkey[wv * 64 * R + h * 64 + lane] = k[h];
                    bidx[wv * 64 * R + h * 64 + lane] = x[h];
                }
                __syncthreads();
#pragma unroll
                for (int h = 0; h < R; ++h) {
                    const int e = wv * 64 * R + h * 64 + lane;
                    const uint64_t pk = bkey[e ^ j];
                    const uint32_t px = bidx[e ^ j];
                    const bool keep_earlier = ((e & j) == 0) == ((e & kk) == 0);
                    if (keep_earlier != before(k[h], x[h], pk, px)) { k[h] = pk; x[h] = px; }
                }
            } else if (j >= 64) {
                // partner in the same lane: register h ^ (j / 64); the lower one is h
                const int hj = j >> 6;
#pragma unroll
                for (int h = 0; h < R; ++h) {
                    int h2 = -1;
                    if constexpr (R >= 2) { if (hj == 1 && (h & 1) == 0) h2 = h + 1; }
                    if constexpr (R >= 4) { if (hj == 2 && (h & 2) == 0) h2 = h + 2; }
                    if (h2 < 0) continue;
#pragma unroll
                    for (int g = 1; g < R; ++g) {
                        if (g != h2) continue;
                        const int e = wv * 64 * R + h * 64 + lane;
                        const bool up = (e & kk) == 0;
                        // up: h keeps the earlier, g the later; otherwise the reverse
                        if (up != before(k[h], x[h], k[g], x[g])) {
                            const uint64_t tk = k[h]; k[h] = k[g]; k[g] = tk;
                            const uint32_t tx = x[h]; x[h] = x[g]; x[g] = tx;
                        }
                    }
                }
            } else {
                // partner lane ^ j of the same register
#pragma unroll
                for (int h = 0; h < R; ++h) {
                    const int e = wv * 64 * R + h * 64 + lane;
                    const uint64_t pk = __shfl_xor(k[h], j, 64);
                    const uint32_t px = (uint32_t)__shfl_xor((int)x[h], j, 64);
                    const bool keep_earlier = ((e & j) == 0) == ((e & kk) == 0);
                    if (keep_earlier != before(k[h], x[h], pk, px)) { k[h] = pk; x[h] = px; }
                }
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int h = 0; h < R; ++h) {
        bkey[wv * 64 * R + h * 64 + lane] = k[h];
        bidx[wv * 64 * R + h * 64 + lane] = x[h];
    }
    __syncthreads();
}

// Calls f(key, i) for every candidate i of the list, thread tid taking i = tid, tid + 1024, ...
// Eight key loads per thread are issued before any is used, so a pass is not a chain of dependent
// global-memory latencies. The pixel indices are read by f only where it needs them.
template <typename F>
__device__ __forceinline__ void for_each_key(const uint64_t* keys, uint32_t N, int tid, F f)
{
    constexpr int UNR = 8;
    for (uint32_t i0 = tid; i0 < N; i0 += 1024 * UNR) {
        // the loads are issued unconditionally (indices past the list read its last entry, i0 < N)
        // so that no branch separates them
        uint64_t kb[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u) kb[u] = keys[min(i0 + 1024u * u, N - 1)];
#pragma unroll
        for (int u = 0; u < UNR; ++u)
            if (i0 + 1024u * u < N) f(kb[u], i0 + 1024u * u);
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
    // accepted corners (x, y); the scan below reads 4 at a time, up to 2 x 64 + 3 entries past the last
    __shared__ __attribute__((aligned(16))) int2 acc_xy[VS_MAX_CORNERS + 2 * 64 + 4];
    __shared__ __attribute__((aligned(16))) int2 bxy[CAP];   // (x, y) of the sorted batch
    __shared__ uint32_t s_conf[64];
    __shared__ uint64_t s_mask[64];
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
    const uint32_t d2_32 = d2 < 0xFFFFFFFFll ? (uint32_t)d2 : 0xFFFFFFFFu;

    if (tid == 0) { s_nacc = 0; s_done = !(lmax > 0.0) || K <= 0; }
    __syncthreads();

    // keys requested per batch: the greedy typically consumes about 1.2 K candidates, so 1.5 K keeps
    // one batch (and a 2048-element sort for K up to ~1300) in the common case
    const uint32_t batch = (uint32_t)min(BATCH, max(512, K + K / 2));
    const uint64_t span = lmax_bits >= base ? lmax_bits - base : 0;
    const int nbits = (span ? 64 - __clzll((long long)span) : 0) + 32;
    bool unbounded = true;
    u128 U = 0;                    // exclusive upper bound on composite keys still to process

    // ---- 0) the first batch's cut from the score histogram the response kernel built (suffix sums
    // over its bins): the highest bin above the threshold's from which on at least `batch` scores lie,
    // when they fit the batch buffer; all eligible scores when the bins above the threshold's hold
    // fewer and they fit. Otherwise, and for later batches, the radix select below.
    __shared__ int s_cut_ok;
    __shared__ unsigned long long s_cut;
    {
        constexpr int NS = 1024;
        static_assert(NBIN_S <= NS && NS <= 1024 && NS <= NBIN, "histogram scan size");
        const uint32_t* hh = hist_of(ws, item_bytes, item);
        if (tid < NS) hist[tid] = tid < NBIN_S ? hh[tid] : 0u;
        if (tid == 0) { s_cut_ok = 0; s_cut = 0; }
        __syncthreads();
        for (int o = 1; o < NS; o <<= 1) {
            const uint32_t add = (tid < NS && tid + o < NS) ? hist[tid + o] : 0u;
            __syncthreads();
            if (tid < NS) hist[tid] += add;
            __syncthreads();
        }
        // hist[b] now counts the scores in bins >= b
        const int bb = score_bin(base);
        if (tid > bb && tid < NBIN_S) {
            const uint32_t sfx = hist[tid], nxt = tid + 1 < NS ? hist[tid + 1] : 0u;
            if (sfx >= batch && nxt < batch && sfx <= CAP) {   // at most one bin qualifies
                s_cut_ok = 1;
                s_cut = bin_low(tid) - base;
            }
        }
        if (tid == 0 && (bb + 1 < NS ? hist[bb + 1] : 0u) < batch && hist[bb] <= CAP) s_cut_ok = 1;   // T = 0
        __syncthreads();
    }
    bool first = true;

    while (!s_done) {
        // ---- 1) radix select the cut T: all eligible keys in [T, U) form the batch. The first digit
        // pass also counts the eligible keys: none left ends the selection, and when they all fit the
        // batch is all of them (T = 0).
        u128 T = 0;
        bool none_left = false;
        const bool from_hist = first && s_cut_ok;
        first = false;
        if (from_hist) {
            T = (u128)s_cut << 32;
        } else {
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
                // most keys fall into a few low bins: the lanes sharing the first active lane's bin
                // add in one atomic, the others one each
                auto add_bin = [&](bool in, uint32_t b) {
                    const uint32_t b0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)b);
                    const uint64_t same = __ballot(in && b == b0);
                    if (same && lane == (int)__builtin_ctzll(same)) atomicAdd(&hist[b0], (uint32_t)__popcll(same));
                    if (in && b != b0) atomicAdd(&hist[b], 1u);
                };
                const uint32_t dmask = (1u << db) - 1u;
                if (unbounded && shift >= 32) {
                    // the digit and the prefix lie in the score bits: 64-bit arithmetic on them
                    const int ps = pshift - 32, ds = shift - 32;   // ps <= 63: the span has at most 63 bits
                    const uint64_t pre = (uint64_t)prefix;
                    for_each_key(keys, N, tid, [&](uint64_t kb, uint32_t) {
                        const uint64_t vk = kb - base;
                        const bool in = kb >= base && (vk >> ps) == pre;
                        add_bin(in, in ? (uint32_t)(vk >> ds) & dmask : 0xFFFFFFFFu);
                    });
                } else {
                    for_each_key(keys, N, tid, [&](uint64_t kb, uint32_t i) {
                        bool in = kb >= base;
                        u128 v = 0;
                        if (in) {
                            // the index (the composite key's low 32 bits) matters only when this digit
                            // reaches into it or the score bits tie with the bound U's
                            const bool need_ix = shift < 32 || (!unbounded && kb - base == (uint64_t)(U >> 32));
                            v = comp(kb, need_ix ? idx[i] : 0u, base);
                            in = (unbounded || v < U) && !(pshift < 128 && (v >> pshift) != prefix);
                        }
                        add_bin(in, in ? ((uint32_t)(v >> shift) & dmask) : 0xFFFFFFFFu);
                    });
                }
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

        // ---- 2) gather [T, U) into LDS: the score bits decide, except where they tie with T's or U's
        // and the bound's index bits are not zero; then the key's index is read. Each gathered key
        // records its list position, replaced by its pixel index once the pass is over (one round of
        // loads instead of a load latency inside the pass).
        if (tid == 0) s_bcount = 0;
        __syncthreads();
        {
            const uint64_t Tk = (uint64_t)(T >> 32), Uk = (uint64_t)(U >> 32);
            const uint32_t Tlo = (uint32_t)T, Ulo = (uint32_t)U;
            for_each_key(keys, N, tid, [&](uint64_t kb, uint32_t i) {
                bool take = kb >= base;
                if (take) {
                    const uint64_t vk = kb - base;
                    take = vk >= Tk && (unbounded || vk < Uk);
                    const bool need_ix = (vk == Tk && Tlo != 0u) || (!unbounded && vk == Uk && Ulo != 0u);
                    if (need_ix) {
                        const u128 v = comp(kb, idx[i], base);
                        take = !(v < T || (!unbounded && v >= U));
                    }
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
                    bidx[slot] = i;
                }
            });
        }
        __syncthreads();
        for (int s2 = tid; s2 < min((int)s_bcount, CAP); s2 += 1024) bidx[s2] = idx[bidx[s2]];
        __syncthreads();
        const int bc = s_bcount < CAP ? s_bcount : CAP;
        // the batch is padded with entries that order last to the sorting size 1024, 2048 or 4096
        const int ssize = bc <= 1024 ? 1024 : (bc <= 2048 ? 2048 : 4096);
        for (int i = bc + tid; i < ssize; i += 1024) { bkey[i] = 0; bidx[i] = 0xFFFFFFFFu; }
        __syncthreads();

        // ---- 3) bitonic sort, earliest first
        if (ssize == 1024)
            sort_batch<1>(bkey, bidx, tid);
        else if (ssize == 2048)
            sort_batch<2>(bkey, bidx, tid);
        else
            sort_batch<4>(bkey, bidx, tid);

        // ---- 4) greedy acceptance, 64 candidates at a time. The batch's coordinates are formed in
        // parallel first. Per group, all waves test the members against the corners accepted so far
        // and mark, per member, the earlier members of the group that are too close (one bit each).
        // Wave 0 then accepts the members clear of both at once and walks only the contested ones in
        // order. Two barriers a group.
        for (int i = tid; i < bc; i += 1024) {
            const uint32_t ix = bidx[i];
            bxy[i] = make_int2((int32_t)(ix % (uint32_t)W), (int32_t)(ix / (uint32_t)W));
        }
        if (tid < 64) {
            s_conf[tid] = 0;
            s_mask[tid] = 0;
        }
        __syncthreads();
        for (int g0 = 0; g0 < bc; g0 += 64) {
            const int na = s_nacc;
            if (na >= K) break;
            const int gn = min(64, bc - g0);                  // members in this group
            if (W <= D24_MAX_SIDE && H <= D24_MAX_SIDE)
                greedy_test<true>(bxy, acc_xy, g0, gn, na, lane, wv, d2_32, d2, s_conf, s_mask);
            else
                greedy_test<false>(bxy, acc_xy, g0, gn, na, lane, wv, d2_32, d2, s_conf, s_mask);
            __syncthreads();
            if (wv == 0) {
                const bool valid = lane < gn;
                const int2 c = valid ? bxy[g0 + lane] : make_int2(0, 0);
                const bool pre_ok = valid && s_conf[lane] == 0;
                const uint64_t ok = __ballot(pre_ok);
                const uint64_t mask = s_mask[lane] & ok;      // earlier members still eligible and too close
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
                    acc_xy[rank] = c;
                    float* o = xy_out + rank * 2;
                    o[0] = (float)c.x;
                    o[1] = (float)c.y;
                    if (score_out) score_out[rank] = __longlong_as_double((long long)bkey[g0 + lane]);
                }
                if (lane == 0) s_nacc = na + min(__popcll(acc), allowed);
                s_conf[lane] = 0;
                s_mask[lane] = 0;
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

// the three detection launches over n items
template <class IO>
int launch_detect(const IO& io, int n, int width, int height, int pitch, const vs_detect_params& p, int Kmax,
                  int capacity, uint8_t* w8, hipStream_t s)
{
    const int64_t ib = per_item_bytes(width, height);
    detect_init_kernel<<<n, 256, 0, s>>>(w8, ib, n, io);
    int e = vs::check_launch("vs_detect_corners(init)");
    if (e) return e;
    const int rw = width - 2 * p.roi_mx, rh = height - 2 * p.roi_my;
    // each output row belongs to one wave's segment and the candidates are sorted afterwards, so the
    // segment height only trades per-wave warm-up rows against waves per frame
    const int sr = vs::detect_segment_rows(n, SR_FEW, SR);
    const int strips = (rw + SW - 1) / SW, segs = (rh + sr - 1) / sr;
    const int64_t nwaves = (int64_t)n * strips * segs;
    corner_response_kernel<<<(unsigned)((nwaves + RESP_WAVES - 1) / RESP_WAVES), 64 * RESP_WAVES, 0, s>>>(
        io, width, height, pitch, p.roi_mx, p.roi_my, n, strips, segs, sr, w8, ib);
    e = vs::check_launch("vs_detect_corners(response)");
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
