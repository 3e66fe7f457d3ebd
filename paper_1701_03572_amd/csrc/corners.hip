// detect_corners: Shi-Tomasi response + 3x3 NMS over the ROI, then the ordered greedy top-K.
//
// Kernel 1 (corner_response): one 256-thread workgroup per 128x16 ROI tile stages the pixels with
// a 3-pixel halo in LDS, forms Sobel gradients and 3x3 box sums of the tensor (exact int32), and
// keeps the 3x3 local maxima inside the ROI. The NMS runs on an FP32 estimate of the score with
// a bounded relative error; a comparison that falls inside the error band, and every survivor,
// uses the exact binary64 score 2 det / (tr + sqrt(disc)) from exact det/tr/disc, so the result
// is the exact-score NMS. Survivors are appended (block-compacted, one atomic per workgroup) to
// the item's candidate list in the workspace; the item's maximum score is folded in with an
// integer atomic max on the score's bit pattern (non-negative doubles order like their bits).
//
// Kernel 2 (corner_select): one 1024-thread workgroup per item. Candidates below
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
    uint32_t count;
    uint32_t pad;
    uint64_t lmax_bits;
};

constexpr int64_t HDR = 256;
constexpr int RTW = 128;        // response tile width (rows of ~one cache line)
constexpr int RTH = 16;         // response tile height
constexpr int PER_T = RTW * RTH / 256;   // pixels per thread in the NMS pass
constexpr int PTW = RTW + 6, PTH = RTH + 6;   // pixel tile with 3-pixel halo
constexpr int GTW = RTW + 4, GTH = RTH + 4;   // gradient tile (halo 2)
constexpr int LTW = RTW + 2, LTH = RTH + 2;   // score tile (halo 1)
constexpr int CAP = 4096;       // LDS batch capacity of the selection
constexpr int BATCH = 2048;     // keys requested per batch
constexpr int DIGIT = 11;
constexpr int NBIN = 1 << DIGIT;

__host__ __device__ inline int64_t per_item_bytes(int w, int h)
{
    const int64_t c = (int64_t)w * h;
    return (HDR + 8 * c + 4 * c + 255) & ~(int64_t)255;
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

__device__ __forceinline__ bool gated_off(const int32_t* gate, int gate_min, int64_t rec)
{
    return gate != nullptr && gate[rec] >= gate_min;
}

__global__ void detect_init_kernel(uint8_t* ws, int64_t item_bytes, int n, int istride, const int32_t* gate,
                                   int gate_min)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || gated_off(gate, gate_min, (int64_t)i * istride)) return;
    CandHeader* h = hdr_of(ws, item_bytes, i);
    h->count = 0;
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

// FP32 estimate of the same score, relative error below 5e-7 (each of the roughly ten rounded
// steps contributes at most one or two units of 2^-24); 0 exactly when det == 0.
__device__ __forceinline__ float approx_key(int32_t A, int32_t B, int32_t C)
{
    const double a = (double)A, b = (double)B, c = (double)C;
    const double det = a * c - b * b;
    if (!(det > 0.0)) return 0.0f;
    const double dm = a - c;
    const double disc = dm * dm + 4.0 * (b * b);
    const float sf = __builtin_amdgcn_sqrtf((float)disc);
    return 2.0f * (float)det * __builtin_amdgcn_rcpf((float)(a + c) + sf);
}

// half-width of the band inside which two FP32 estimates are compared exactly
constexpr float KEY_BAND = 1e-5f;

__device__ __forceinline__ void box_tensor(const int16_t (*gxs)[GTW], const int16_t (*gys)[GTW], int r, int c, int32_t& A,
                                           int32_t& B, int32_t& C)
{
    A = B = C = 0;
#pragma unroll
    for (int dy = 0; dy < 3; ++dy)
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) {
            const int32_t gx = gxs[r + dy][c + dx], gy = gys[r + dy][c + dx];
            A += gx * gx;
            B += gx * gy;
            C += gy * gy;
        }
}

__global__ __launch_bounds__(256) void corner_response_kernel(const uint8_t* __restrict__ frames, int64_t frame_stride,
                                                              int W, int H, int pitch, int mx, int my,
                                                              int n_items, int tiles_x, int tiles_y, int by_xcd,
                                                              int istride, const int32_t* gate, int gate_min,
                                                              uint8_t* ws, int64_t item_bytes)
{
    int item, tile;
    if (!vs::xcd_map(blockIdx.x, n_items, tiles_x * tiles_y, by_xcd != 0, item, tile)) return;
    if (gated_off(gate, gate_min, (int64_t)item * istride)) return;
    __shared__ uint8_t pix[PTH][PTW + 2];
    __shared__ int16_t gxs[GTH][GTW];
    __shared__ int16_t gys[GTH][GTW];
    __shared__ float lam[LTH][LTW + 1];       // FP32 score estimates; -1 outside the ROI
    __shared__ uint32_t wave_cnt[4];
    __shared__ uint64_t wave_max[4];
    __shared__ uint32_t block_base;

    const uint8_t* img = frames + item * frame_stride;
    const int rx0 = mx, ry0 = my, rx1 = W - mx, ry1 = H - my;
    const int tyi = tile / tiles_x, txi = tile - tyi * tiles_x;
    const int tx0 = rx0 + txi * RTW, ty0 = ry0 + tyi * RTH;
    const int tid = threadIdx.x;

    // pixels needed by in-ROI scores lie in [rx0-2, rx1+2) x [ry0-2, ry1+2), inside the image
    for (int k = tid; k < PTH * PTW; k += 256) {
        const int r = k / PTW, c = k - r * PTW;
        const int x = tx0 - 3 + c, y = ty0 - 3 + r;
        uint8_t v = 0;
        if (x >= rx0 - 2 && x < rx1 + 2 && y >= ry0 - 2 && y < ry1 + 2) v = img[(int64_t)y * pitch + x];
        pix[r][c] = v;
    }
    __syncthreads();
    for (int k = tid; k < GTH * GTW; k += 256) {
        const int r = k / GTW, c = k - r * GTW;   // gradient at pixel-tile (r + 1, c + 1)
        const int pr = r + 1, pc = c + 1;
        const int gx = (pix[pr - 1][pc + 1] - pix[pr - 1][pc - 1]) + 2 * (pix[pr][pc + 1] - pix[pr][pc - 1]) +
                       (pix[pr + 1][pc + 1] - pix[pr + 1][pc - 1]);
        const int gy = (pix[pr + 1][pc - 1] - pix[pr - 1][pc - 1]) + 2 * (pix[pr + 1][pc] - pix[pr - 1][pc]) +
                       (pix[pr + 1][pc + 1] - pix[pr - 1][pc + 1]);
        gxs[r][c] = (int16_t)gx;
        gys[r][c] = (int16_t)gy;
    }
    __syncthreads();
    for (int k = tid; k < LTH * LTW; k += 256) {
        const int r = k / LTW, c = k - r * LTW;   // score at gradient-tile (r + 1, c + 1)
        const int x = tx0 - 1 + c, y = ty0 - 1 + r;
        float v = -1.0f;                           // outside the ROI: ignored by the NMS
        if (x >= rx0 && x < rx1 && y >= ry0 && y < ry1) {
            int32_t A, B, C;
            box_tensor(gxs, gys, r, c, A, B, C);
            v = approx_key(A, B, C);
        }
        lam[r][c] = v;
    }
    __syncthreads();

    // 3x3 NMS on the estimates; comparisons inside the band are redone with exact keys. Thread t
    // owns tile row t / 16 and columns (t % 16) + 16 q, so neighbouring lanes read neighbouring
    // words of the score tile.
    const int pr = tid >> 4, pcol = tid & 15;
    uint32_t mine = 0;
    uint64_t my_max = 0;
    uint32_t my_idx[PER_T];
    uint64_t my_key[PER_T];
#pragma unroll
    for (int q = 0; q < PER_T; ++q) {
        const int c = pcol + 16 * q;
        const int x = tx0 + c, y = ty0 + pr;
        const float v = lam[pr + 1][c + 1];
        if (x >= rx1 || y >= ry1 || !(v > 0.0f)) continue;
        const float hi = v * (1.0f + KEY_BAND), lo = v * (1.0f - KEY_BAND);
        bool beaten = false;
        uint32_t close = 0;                        // neighbours whose estimate is inside the band
#pragma unroll
        for (int dy = 0; dy < 3; ++dy)
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) {
                if (dy == 1 && dx == 1) continue;
                const float u = lam[pr + dy][c + dx];
                if (u > hi) beaten = true;
                else if (u >= lo) close |= 1u << (dy * 3 + dx);
            }
        if (beaten) continue;
        int32_t A, B, C;
        box_tensor(gxs, gys, pr + 1, c + 1, A, B, C);
        const double key = exact_key(A, B, C);
        while (close) {
            const int bit = __ffs(close) - 1;
            close &= close - 1;
            const int dy = bit / 3, dx = bit - dy * 3;
            box_tensor(gxs, gys, pr + dy, c + dx, A, B, C);
            if (exact_key(A, B, C) > key) beaten = true;
        }
        if (beaten) continue;
        const uint64_t kb = (uint64_t)__double_as_longlong(key);
        my_max = kb > my_max ? kb : my_max;
        my_key[mine] = kb;
        my_idx[mine] = (uint32_t)(y * W + x);
        ++mine;
    }
    // block exclusive scan of the per-thread counts, and the block max (the maximum score of the
    // ROI is always a local maximum, so the maximum over survivors is the ROI maximum)
    const int lane = tid & 63, wv = tid >> 6;
    uint32_t incl = mine;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t t = __shfl_up(incl, o, 64);
        if (lane >= o) incl += t;
    }
    uint64_t wmax = my_max;
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        const uint64_t t = __shfl_xor(wmax, m, 64);
        wmax = t > wmax ? t : wmax;
    }
    if (lane == 63) wave_cnt[wv] = incl;
    if (lane == 0) wave_max[wv] = wmax;
    __syncthreads();
    if (tid == 0) {
        const uint32_t tot = wave_cnt[0] + wave_cnt[1] + wave_cnt[2] + wave_cnt[3];
        CandHeader* h = hdr_of(ws, item_bytes, item);
        block_base = tot ? atomicAdd(&h->count, tot) : 0u;
        uint64_t bm = wave_max[0];
        for (int i = 1; i < 4; ++i) bm = wave_max[i] > bm ? wave_max[i] : bm;
        if (bm) atomicMax((unsigned long long*)&h->lmax_bits, (unsigned long long)bm);
    }
    __syncthreads();
    uint32_t base = block_base + incl - mine;
    for (int i = 0; i < wv; ++i) base += wave_cnt[i];
    uint64_t* keys = keys_of(ws, item_bytes, item);
    uint32_t* idx = idx_of(ws, item_bytes, item, W, H);
    for (uint32_t q = 0; q < mine; ++q) {
        keys[base + q] = my_key[q];
        idx[base + q] = my_idx[q];
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

__global__ __launch_bounds__(1024) void corner_select_kernel(uint8_t* ws, int64_t item_bytes, int W, int H,
                                                             int istride, const int32_t* gate, int gate_min, int K,
                                                             double quality, int min_dist, int capacity,
                                                             float* __restrict__ xy_out, double* __restrict__ score_out,
                                                             int32_t* __restrict__ count_out,
                                                             uint8_t* __restrict__ alive_out)
{
    const int item = blockIdx.x;
    const int64_t rec = (int64_t)item * istride;
    if (gated_off(gate, gate_min, rec)) return;
    __shared__ uint64_t bkey[CAP];
    __shared__ uint32_t bidx[CAP];
    __shared__ uint32_t hist[NBIN];
    __shared__ int32_t acc_x[VS_MAX_CORNERS];
    __shared__ int32_t acc_y[VS_MAX_CORNERS];
    __shared__ uint32_t s_conf[64];
    __shared__ int32_t s_cx[64], s_cy[64];
    __shared__ int s_nacc, s_bcount, s_digit, s_done;
    __shared__ uint32_t s_need, s_above, s_sel_in_bin;
    __shared__ uint32_t s_red[32];

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

    const uint64_t span = lmax_bits >= base ? lmax_bits - base : 0;
    const int nbits = (span ? 64 - __clzll((long long)span) : 0) + 32;
    bool unbounded = true;
    u128 U = 0;                    // exclusive upper bound on composite keys still to process

    while (!s_done) {
        // ---- 1) count the eligible keys below U
        uint32_t cnt = 0;
        for (uint32_t i = tid; i < N; i += 1024) {
            const uint64_t kb = keys[i];
            if (kb < base) continue;
            if (!unbounded && comp(kb, idx[i], base) >= U) continue;
            ++cnt;
        }
        cnt = (uint32_t)vs::wave_sum_i((int)cnt);
        if (lane == 0) s_red[wv] = cnt;
        __syncthreads();
        uint32_t n_elig = 0;
        for (int i = 0; i < 16; ++i) n_elig += s_red[i];
        __syncthreads();
        if (n_elig == 0) break;

        // ---- 2) radix select the cut T: all eligible keys in [T, U) form the batch
        u128 T = 0;
        if (n_elig > CAP) {
            int shift = nbits;
            u128 prefix = 0;
            if (tid == 0) { s_need = BATCH; s_above = 0; }
            __syncthreads();
            while (true) {
                const int db = shift < DIGIT ? shift : DIGIT;
                const int pshift = shift;             // prefix covers bits >= pshift
                shift -= db;
                for (int b = tid; b < NBIN; b += 1024) hist[b] = 0;
                __syncthreads();
                for (uint32_t i = tid; i < N; i += 1024) {
                    const uint64_t kb = keys[i];
                    if (kb < base) continue;
                    const u128 v = comp(kb, idx[i], base);
                    if (!unbounded && v >= U) continue;
                    if (pshift < 128 && (v >> pshift) != prefix) continue;
                    atomicAdd(&hist[(uint32_t)(v >> shift) & ((1u << db) - 1u)], 1u);
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
                // hist[b] is now the count of keys with digit >= b
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

        // ---- 3) gather [T, U) into LDS
        if (tid == 0) s_bcount = 0;
        __syncthreads();
        for (uint32_t i = tid; i < N; i += 1024) {
            const uint64_t kb = keys[i];
            if (kb < base) continue;
            const uint32_t ix = idx[i];
            const u128 v = comp(kb, ix, base);
            if (v < T || (!unbounded && v >= U)) continue;
            const int slot = atomicAdd(&s_bcount, 1);
            if (slot < CAP) {          // always true by construction of T; keeps LDS writes in range
                bkey[slot] = kb;
                bidx[slot] = ix;
            }
        }
        __syncthreads();
        const int bc = s_bcount < CAP ? s_bcount : CAP;
        int p2 = 1;
        while (p2 < bc) p2 <<= 1;
        for (int i = bc + tid; i < p2; i += 1024) { bkey[i] = 0; bidx[i] = 0xFFFFFFFFu; }
        __syncthreads();

        // ---- 4) bitonic sort, earliest first
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

        // ---- 5) greedy acceptance, 64 candidates at a time
        for (int g0 = 0; g0 < bc; g0 += 64) {
            const int na = s_nacc;
            if (na >= K) break;
            if (tid < 64) {
                s_conf[tid] = 0;
                if (g0 + tid < bc) {
                    const uint32_t ix = bidx[g0 + tid];
                    s_cx[tid] = (int32_t)(ix % (uint32_t)W);
                    s_cy[tid] = (int32_t)(ix / (uint32_t)W);
                }
            }
            __syncthreads();
            if (g0 + lane < bc) {
                const int cx = s_cx[lane], cy = s_cy[lane];
                bool conf = false;
                for (int j = wv; j < na; j += 16) {
                    const int64_t dx = cx - acc_x[j], dy = cy - acc_y[j];
                    if (dx * dx + dy * dy < d2) { conf = true; break; }
                }
                if (conf) s_conf[lane] = 1;
            }
            __syncthreads();
            if (wv == 0) {
                const bool valid = g0 + lane < bc;
                const int cx = valid ? s_cx[lane] : 0, cy = valid ? s_cy[lane] : 0;
                uint64_t mask = 0;                      // earlier group members too close
                for (int k = 0; k < 64; ++k) {
                    if (k >= lane || g0 + k >= bc) break;
                    const int64_t dx = cx - s_cx[k], dy = cy - s_cy[k];
                    if (dx * dx + dy * dy < d2) mask |= 1ull << k;
                }
                const uint32_t pre = valid ? s_conf[lane] : 1u;
                uint64_t acc_mask = 0;
                int cnt_acc = na;
                for (int k = 0; k < 64; ++k) {
                    const uint32_t pk = __builtin_amdgcn_readlane(pre, k);
                    const uint32_t mlo = __builtin_amdgcn_readlane((uint32_t)mask, k);
                    const uint32_t mhi = __builtin_amdgcn_readlane((uint32_t)(mask >> 32), k);
                    const uint64_t mk = ((uint64_t)mhi << 32) | mlo;
                    if (!pk && !(mk & acc_mask) && cnt_acc < K) {
                        acc_mask |= 1ull << k;
                        ++cnt_acc;
                    }
                }
                if ((acc_mask >> lane) & 1ull) {
                    const int rank = na + __popcll(acc_mask & ((1ull << lane) - 1ull));
                    acc_x[rank] = cx;
                    acc_y[rank] = cy;
                    float* o = xy_out + (rec * capacity + rank) * 2;
                    o[0] = (float)cx;
                    o[1] = (float)cy;
                    if (score_out)
                        score_out[rec * capacity + rank] = __longlong_as_double((long long)bkey[g0 + lane]);
                }
                if (lane == 0) s_nacc = cnt_acc;
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
    for (int k = tid; k < capacity; k += 1024) alive_out[rec * capacity + k] = k < na ? 1 : 0;
    if (tid == 0) count_out[rec] = na;
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
    if (n < 0 || istride < 1 || width < 8 || height < 8 || pitch < width)
        return vs::set_error(VS_ERR_INVALID, "vs_detect_corners: bad size");
    if (capacity > VS_MAX_CORNERS) return vs::set_error(VS_ERR_UNSUPPORTED, "vs_detect_corners: capacity > %d", VS_MAX_CORNERS);
    if (p->max_corners < 0 || p->max_corners > capacity || capacity <= 0)
        return vs::set_error(VS_ERR_INVALID, "vs_detect_corners: need 0 <= max_corners <= capacity");
    if (p->roi_mx < 2 || p->roi_my < 2 || width - 2 * p->roi_mx <= 0 || height - 2 * p->roi_my <= 0)
        return vs::set_error(VS_ERR_INVALID, "vs_detect_corners: ROI margins must be >= 2 and leave a non-empty ROI");
    if (p->min_dist < 0 || !(p->quality >= 0.0) || p->quality > 1.0)
        return vs::set_error(VS_ERR_INVALID, "vs_detect_corners: bad min_dist or quality");
    if (n == 0) return VS_OK;
    if (n > 65535) return vs::set_error(VS_ERR_INVALID, "vs_detect_corners: more than 65535 items");
    if (n > 1 && frame_stride < (int64_t)pitch * height)
        return vs::set_error(VS_ERR_INVALID, "vs_detect_corners: frame stride overlaps items");
    if ((int64_t)width * height >= (int64_t)1 << 32)
        return vs::set_error(VS_ERR_UNSUPPORTED, "vs_detect_corners: frame too large");
    const size_t need = vs_detect_workspace(width, height, n);
    if (ws_bytes < need) return vs::set_error(VS_ERR_WORKSPACE, "vs_detect_corners: workspace %zu < %zu", ws_bytes, need);
    if (reinterpret_cast<uintptr_t>(workspace) & 255)
        return vs::set_error(VS_ERR_INVALID, "vs_detect_corners: workspace must be 256-byte aligned");
    hipStream_t s = vs::as_stream(stream);
    const int64_t ib = per_item_bytes(width, height);
    uint8_t* w8 = static_cast<uint8_t*>(workspace);
    detect_init_kernel<<<(n + 255) / 256, 256, 0, s>>>(w8, ib, n, istride, gate, gate_min);
    int e = vs::check_launch("vs_detect_corners(init)");
    if (e) return e;
    const int rw = width - 2 * p->roi_mx, rh = height - 2 * p->roi_my;
    const int tiles_x = (rw + RTW - 1) / RTW, tiles_y = (rh + RTH - 1) / RTH;
    const bool by_xcd = n >= VS_XCD_MIN_ITEMS;
    const int64_t nblk = vs::xcd_grid(n, tiles_x * tiles_y, by_xcd);
    corner_response_kernel<<<(unsigned)nblk, 256, 0, s>>>(frames, frame_stride, width, height, pitch, p->roi_mx,
                                                          p->roi_my, n, tiles_x, tiles_y, by_xcd, istride, gate,
                                                          gate_min, w8, ib);
    e = vs::check_launch("vs_detect_corners(response)");
    if (e) return e;
    corner_select_kernel<<<n, 1024, 0, s>>>(w8, ib, width, height, istride, gate, gate_min, p->max_corners, p->quality,
                                            p->min_dist, capacity, xy, score, count, alive);
    return vs::check_launch("vs_detect_corners(select)");
}
