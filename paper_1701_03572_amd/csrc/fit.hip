// fit_similarity / fit_motion: seeded robust rigid / similarity / affine fit, hybrid dwell switch
// and skip rule.
//
// Kernel 1a (fit_hyp): the RANSAC hypotheses of each pair, spread over up to 8 workgroups per pair
// when there are few pairs; each records its best. Kernel 1b (fit_pair): one 256-thread workgroup
// per pair, with LDS sized to the capacity (19 bytes per point slot) and registers capped for three
// workgroups per CU, so pairs overlap each other's LDS and FP64 latencies. The valid slots are
// compacted in slot order into LDS (raw FP32 coordinates, centred exactly in binary64 when read),
// then each requested model is fitted:
// the hypothesis workgroups' waves share the RANSAC hypotheses (wave w of workgroup s of S takes
// h = s + S (w + 4k)), score them by
// counting residuals <= threshold with a wave reduction, and the best (most inliers, then
// smallest h) is refitted by least squares in binary64: the similarity through its 4x4 normal
// equations (Gaussian elimination with partial pivoting), the rigid model through the centred
// closed form atan2, the affine through its centroids and the centred 2x2 second moments.
// Fixed-order reductions keep the result independent of scheduling. The hypotheses (2-point
// similarity / rigid, 3-point affine) and residuals use exactly the operation order
//     px = (ar x - ai y) + br,  py = (ai x + ar y) + bi          (similarity, rigid)
//     px = (a11 x + a12 y) + tx,  py = (a21 x + a22 y) + ty      (affine)
//     d2 = dx dx + dy dy
// with floating-point contraction disabled, so inlier decisions are bit-reproducible.
// Kernel 2 (fit_resolve): the dwell-block state machine over the pairs of the call, evaluated
// block-parallel. Kernel 3 (fit_emit): one workgroup per pair writes the chosen model's parameters,
// info and inlier flags.
#include <algorithm>
#include <cmath>
#include <mutex>

#include "vs_common.hpp"

#pragma clang fp contract(off)

namespace {

struct ModelFit {
    double p[6];     // (a, b, tx, ty) for rigid / similarity; (a11, a12, tx, a21, a22, ty) for the affine
    double err;
    int32_t n_inl;
    int32_t pad;
};

constexpr int N_SLOTS = 3;
__host__ __device__ inline int slot_of_model(int model) { return model == VS_AFFINE ? 2 : model; }

struct PairRec {
    int32_t n_valid;
    int32_t skipped;
    int32_t pad[2];
    ModelFit m[N_SLOTS];   // rigid, similarity, affine
};
static_assert(sizeof(PairRec) <= 256, "pair record header");

// best hypothesis of one hypothesis workgroup for one model (score -1: none)
struct HypRec {
    int32_t score;
    int32_t h;
    double p[6];
    double pad;
};
static_assert(sizeof(HypRec) == 64, "hypothesis record");
constexpr int MAX_SPLIT = 32;   // hypothesis workgroups per pair at most (one hypothesis per wave for 128)

__host__ __device__ inline int64_t cap_aligned(int cap) { return ((int64_t)cap + 255) & ~(int64_t)255; }
__host__ __device__ inline int64_t hyp_offset(int cap) { return 256 + N_SLOTS * cap_aligned(cap); }
__host__ __device__ inline int64_t rec_bytes(int cap) { return hyp_offset(cap) + MAX_SPLIT * N_SLOTS * sizeof(HypRec); }

__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t ctr)
{
    uint64_t z = seed + (ctr + 1u) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t draw(uint64_t seed, int64_t stream_id, int64_t pair, int h, int k)
{
    const uint64_t ctr = (((uint64_t)stream_id & 0xFFFFFull) << 44) | (((uint64_t)pair & 0xFFFFFFFull) << 16) |
                         (((uint64_t)h & 0x7FFFull) << 1) | ((uint64_t)k & 1u);
    return splitmix64_at(seed, ctr);
}

// 3-point draws: bit 15 of the low field set, so with at most 8191 hypotheses they never meet the
// 2-point counters
__device__ __forceinline__ uint64_t draw3(uint64_t seed, int64_t stream_id, int64_t pair, int h, int k)
{
    const uint64_t ctr = (((uint64_t)stream_id & 0xFFFFFull) << 44) | (((uint64_t)pair & 0xFFFFFFFull) << 16) |
                         0x8000u | (((uint64_t)h & 0x1FFFull) << 2) | ((uint64_t)k & 3u);
    return splitmix64_at(seed, ctr);
}

__device__ __forceinline__ double aff_resid2(const double* m, double x, double y, double xd, double yd)
{
    const double px = (m[0] * x + m[1] * y) + m[2];
    const double py = (m[3] * x + m[4] * y) + m[5];
    const double dx = xd - px, dy = yd - py;
    return dx * dx + dy * dy;
}

__device__ __forceinline__ double resid2(double ar, double ai, double br, double bi, double x, double y, double xd,
                                         double yd)
{
    const double px = (ar * x - ai * y) + br;
    const double py = (ai * x + ar * y) + bi;
    const double dx = xd - px, dy = yd - py;
    return dx * dx + dy * dy;
}

constexpr int NT = 256;

struct FitArgs {
    int32_t model;
    int32_t iters;
    double tau2;
    uint64_t seed;
    int64_t stream_id;
    int32_t min_valid;
    int32_t dwell;
    double cx, cy;
};

// deterministic block sum of NV doubles per thread: a butterfly within each wave (every lane gets
// the same bits), then the four wave totals added in a fixed order; every thread gets the total
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* red /* [NV][4] */)
{
    const int t = threadIdx.x, wv = t >> 6;
#pragma unroll
    for (int j = 0; j < NV; ++j) v[j] = vs::wave_sum_d(v[j]);
    if ((t & 63) == 0)
#pragma unroll
        for (int j = 0; j < NV; ++j) red[j * 4 + wv] = v[j];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NV; ++j) v[j] = (red[j * 4] + red[j * 4 + 1]) + (red[j * 4 + 2] + red[j * 4 + 3]);
    __syncthreads();
}

// deterministic block sum of one int per thread (wave sums, then the four in order)
__device__ __forceinline__ int block_sum_i(int v, int* red4)
{
    const int t = threadIdx.x;
    v = vs::wave_sum_i(v);
    if ((t & 63) == 0) red4[t >> 6] = v;
    __syncthreads();
    v = (red4[0] + red4[1]) + (red4[2] + red4[3]);
    __syncthreads();
    return v;
}

// per-pair LDS: the compacted points (4 float arrays), their slots and inlier flags, for a capacity
// rounded up to 64
__host__ __device__ inline int lds_cap(int capacity) { return (capacity + 63) & ~63; }
__host__ __device__ inline size_t pair_lds_bytes(int capacity) { return (size_t)lds_cap(capacity) * 19; }

__device__ void solve4(double A[4][4], double b[4], double x[4])
{
    int perm[4] = {0, 1, 2, 3};
    for (int c = 0; c < 4; ++c) {
        int piv = c;
        for (int r = c + 1; r < 4; ++r)
            if (fabs(A[r][c]) > fabs(A[piv][c])) piv = r;
        if (piv != c) {
            for (int k = 0; k < 4; ++k) { const double t = A[c][k]; A[c][k] = A[piv][k]; A[piv][k] = t; }
            const double t = b[c]; b[c] = b[piv]; b[piv] = t;
            const int tp = perm[c]; perm[c] = perm[piv]; perm[piv] = tp;
        }
        for (int r = c + 1; r < 4; ++r) {
            const double f = A[r][c] / A[c][c];
            for (int k = c; k < 4; ++k) A[r][k] -= f * A[c][k];
            b[r] -= f * b[c];
        }
    }
    for (int r = 3; r >= 0; --r) {
        double s = b[r];
        for (int k = r + 1; k < 4; ++k) s -= A[r][k] * x[k];
        x[r] = s / A[r][r];
    }
    (void)perm;
}

// least squares on the flagged points (all when flags == nullptr); result in out[4]
__device__ __forceinline__ void ls_refit(int model, const float* xs, const float* ys, const float* xd, const float* yd, double cx,
                         double cy, const uint8_t* flags, int n, double* red, double* out)
{
    const int t = threadIdx.x;
    if (model == VS_SIMILARITY) {
        double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};   // n, Sx, Sy, Sx', Sy', S2, Sdot, Scross
        for (int i = t; i < n; i += NT) {
            if (flags && !flags[i]) continue;
            const double x = xs[i] - cx, y = ys[i] - cy, u = xd[i] - cx, w = yd[i] - cy;
            v[0] += 1.0;
            v[1] += x;
            v[2] += y;
            v[3] += u;
            v[4] += w;
            v[5] += x * x + y * y;
            v[6] += x * u + y * w;
            v[7] += x * w - y * u;
        }
        block_sum<8>(v, red);
        if (t == 0) {
            double A[4][4] = {{v[5], 0.0, v[1], v[2]}, {0.0, v[5], -v[2], v[1]}, {v[1], -v[2], v[0], 0.0},
                              {v[2], v[1], 0.0, v[0]}};
            double b[4] = {v[6], v[7], v[3], v[4]};
            double x[4];
            if (v[5] * v[0] - (v[1] * v[1] + v[2] * v[2]) > 0.0) {
                solve4(A, b, x);
            } else {            // all points coincide: pure translation
                x[0] = 1.0;
                x[1] = 0.0;
                x[2] = (v[3] - v[1]) / v[0];
                x[3] = (v[4] - v[2]) / v[0];
            }
            for (int k = 0; k < 4; ++k) out[k] = x[k];
        }
        __syncthreads();
        return;
    }
    // rigid: centroids, then centred cross sums
    double m[5] = {0, 0, 0, 0, 0};
    for (int i = t; i < n; i += NT) {
        if (flags && !flags[i]) continue;
        m[0] += 1.0;
        m[1] += xs[i] - cx;
        m[2] += ys[i] - cy;
        m[3] += xd[i] - cx;
        m[4] += yd[i] - cy;
    }
    block_sum<5>(m, red);
    const double mx = m[1] / m[0], my = m[2] / m[0], mu = m[3] / m[0], mw = m[4] / m[0];
    double s[2] = {0, 0};
    for (int i = t; i < n; i += NT) {
        if (flags && !flags[i]) continue;
        const double x = (xs[i] - cx) - mx, y = (ys[i] - cy) - my, u = (xd[i] - cx) - mu, w = (yd[i] - cy) - mw;
        s[0] += x * u + y * w;
        s[1] += x * w - y * u;
    }
    block_sum<2>(s, red);
    if (t == 0) {
        const double th = atan2(s[1], s[0]);
        const double a = cos(th), b = sin(th);
        out[0] = a;
        out[1] = b;
        out[2] = mu - (a * mx - b * my);
        out[3] = mw - (b * mx + a * my);
    }
    __syncthreads();
}

// affine least squares on the flagged points: centroids, then A = C_uv C_xx^-1 from the centred
// second moments; a singular C_xx (collinear or coincident points) takes the similarity fit.
__device__ __forceinline__ void ls_affine(const float* xs, const float* ys, const float* xd, const float* yd, double cx, double cy,
                          const uint8_t* flags, int n, double* red, double* out6, double* tmp4, int* s_flag)
{
    const int t = threadIdx.x;
    double m[5] = {0, 0, 0, 0, 0};
    for (int i = t; i < n; i += NT) {
        if (flags && !flags[i]) continue;
        m[0] += 1.0;
        m[1] += xs[i] - cx;
        m[2] += ys[i] - cy;
        m[3] += xd[i] - cx;
        m[4] += yd[i] - cy;
    }
    block_sum<5>(m, red);
    const double mx = m[1] / m[0], my = m[2] / m[0], mu = m[3] / m[0], mw = m[4] / m[0];
    double s[7] = {0, 0, 0, 0, 0, 0, 0};   // xx, xy, yy, xu, yu, xw, yw
    for (int i = t; i < n; i += NT) {
        if (flags && !flags[i]) continue;
        const double x = (xs[i] - cx) - mx, y = (ys[i] - cy) - my, u = (xd[i] - cx) - mu, w = (yd[i] - cy) - mw;
        s[0] += x * x;
        s[1] += x * y;
        s[2] += y * y;
        s[3] += x * u;
        s[4] += y * u;
        s[5] += x * w;
        s[6] += y * w;
    }
    block_sum<7>(s, red);
    if (t == 0) {
        const double det = s[0] * s[2] - s[1] * s[1], tr = s[0] + s[2];
        if (det > 1e-12 * tr * tr) {
            out6[0] = (s[3] * s[2] - s[4] * s[1]) / det;
            out6[1] = (s[4] * s[0] - s[3] * s[1]) / det;
            out6[3] = (s[5] * s[2] - s[6] * s[1]) / det;
            out6[4] = (s[6] * s[0] - s[5] * s[1]) / det;
            out6[2] = mu - (out6[0] * mx + out6[1] * my);
            out6[5] = mw - (out6[3] * mx + out6[4] * my);
            *s_flag = 0;
        } else {
            *s_flag = 1;
        }
    }
    __syncthreads();
    if (*s_flag) {
        ls_refit(VS_SIMILARITY, xs, ys, xd, yd, cx, cy, flags, n, red, tmp4);
        if (t == 0) {
            out6[0] = tmp4[0]; out6[1] = -tmp4[1]; out6[2] = tmp4[2];
            out6[3] = tmp4[1]; out6[4] = tmp4[0];  out6[5] = tmp4[3];
        }
        __syncthreads();
    }
}

// Stable compaction of one pair's valid slots into LDS, in slot order: thread t owns a run of
// consecutive slots; an exclusive prefix of the per-thread counts (wave scan, then the wave totals in
// order) places them. Raw FP32 coordinates are stored (centred in binary64 at use, so every side sees
// identical values). Returns the number of valid slots (every thread).
__device__ __forceinline__ int compact_valid(const float* __restrict__ src, const float* __restrict__ dst,
                                             const uint8_t* __restrict__ valid, int64_t base, int capacity, float* xs,
                                             float* ys, float* xd, float* yd, uint16_t* slot_of, int32_t* red4)
{
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int chunk = (capacity + NT - 1) / NT;
    const int c0 = t * chunk, c1 = min(capacity, c0 + chunk);
    int cnt = 0;
    for (int k = c0; k < c1; ++k) cnt += valid[base + k] != 0;
    int incl = cnt;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(incl, o, 64);
        if (lane >= o) incl += y;
    }
    if (lane == 63) red4[wv] = incl;
    __syncthreads();
    int wbase = 0;
    for (int w = 0; w < wv; ++w) wbase += red4[w];
    const int n = (red4[0] + red4[1]) + (red4[2] + red4[3]);
    int o = wbase + incl - cnt;
    for (int k = c0; k < c1; ++k) {
        if (!valid[base + k]) continue;
        xs[o] = src[2 * (base + k)];
        ys[o] = src[2 * (base + k) + 1];
        xd[o] = dst[2 * (base + k)];
        yd[o] = dst[2 * (base + k) + 1];
        if (slot_of) slot_of[o] = (uint16_t)k;
        ++o;
    }
    __syncthreads();
    return n;
}

// The calling wave's best hypothesis of `model` among h = h0, h0 + hs, ... < iters: most inliers,
// the first such h on ties (best = -1, best_h = -1 when none). Every lane returns the same values.
__device__ void ransac_wave(int model, const float* xs, const float* ys, const float* xd, const float* yd, int n,
                            const FitArgs& a, int64_t pair, int h0, int hs, int& best, int& best_h, double (&bm)[6])
{
    const int lane = threadIdx.x & 63;
    const bool affine = model == VS_AFFINE;
    best = -1;
    best_h = -1;
    for (int k = 0; k < 6; ++k) bm[k] = (k == 0 || k == 4) ? 1.0 : 0.0;
    for (int h = h0; h < a.iters; h += hs) {
        double c[6];
        if (affine) {
            const int i1 = (int)(draw3(a.seed, a.stream_id, pair, h, 0) % (uint64_t)n);
            int i2 = (int)(draw3(a.seed, a.stream_id, pair, h, 1) % (uint64_t)n);
            int i3 = (int)(draw3(a.seed, a.stream_id, pair, h, 2) % (uint64_t)n);
            if (i2 == i1) i2 = (i2 + 1) % n;
            while (i3 == i1 || i3 == i2) i3 = (i3 + 1) % n;   // n >= 3: at most two steps
            const double x1 = xs[i1] - a.cx, y1 = ys[i1] - a.cy, u1 = xd[i1] - a.cx, w1 = yd[i1] - a.cy;
            const double ex = (xs[i2] - a.cx) - x1, ey = (ys[i2] - a.cy) - y1;
            const double fx = (xs[i3] - a.cx) - x1, fy = (ys[i3] - a.cy) - y1;
            const double det = ex * fy - fx * ey;
            if (!(fabs(det) >= 1.0)) continue;          // near-collinear sample: no hypothesis
            const double gu = (xd[i2] - a.cx) - u1, gv = (yd[i2] - a.cy) - w1;
            const double hu = (xd[i3] - a.cx) - u1, hv = (yd[i3] - a.cy) - w1;
            c[0] = (gu * fy - hu * ey) / det;
            c[1] = (hu * ex - gu * fx) / det;
            c[3] = (gv * fy - hv * ey) / det;
            c[4] = (hv * ex - gv * fx) / det;
            c[2] = u1 - (c[0] * x1 + c[1] * y1);
            c[5] = w1 - (c[3] * x1 + c[4] * y1);
        } else {
            const int i1 = (int)(draw(a.seed, a.stream_id, pair, h, 0) % (uint64_t)n);
            int i2 = (int)(draw(a.seed, a.stream_id, pair, h, 1) % (uint64_t)n);
            if (i2 == i1) i2 = (i2 + 1) % n;
            const double x1 = xs[i1] - a.cx, y1 = ys[i1] - a.cy, x2 = xs[i2] - a.cx, y2 = ys[i2] - a.cy;
            const double u1 = xd[i1] - a.cx, w1 = yd[i1] - a.cy, u2 = xd[i2] - a.cx, w2 = yd[i2] - a.cy;
            const double dzx = x2 - x1, dzy = y2 - y1;
            const double den = dzx * dzx + dzy * dzy;
            if (den < 1.0) continue;
            const double wx = u2 - u1, wy = w2 - w1;
            double ar = (wx * dzx + wy * dzy) / den;
            double ai = (wy * dzx - wx * dzy) / den;
            double br, bi;
            if (model == VS_RIGID) {
                const double mag = sqrt(ar * ar + ai * ai);
                if (!(mag > 0.0)) continue;
                ar = ar / mag;
                ai = ai / mag;
                const double sxs = x1 + x2, sys = y1 + y2, sxd = u1 + u2, syd = w1 + w2;
                br = (sxd - (ar * sxs - ai * sys)) * 0.5;
                bi = (syd - (ai * sxs + ar * sys)) * 0.5;
            } else {
                br = u1 - (ar * x1 - ai * y1);
                bi = w1 - (ai * x1 + ar * y1);
            }
            c[0] = ar; c[1] = ai; c[2] = br; c[3] = bi; c[4] = 0.0; c[5] = 0.0;
        }
        int sc = 0;
        if (affine) {
            for (int i = lane; i < n; i += 64)
                sc += aff_resid2(c, xs[i] - a.cx, ys[i] - a.cy, xd[i] - a.cx, yd[i] - a.cy) <= a.tau2;
        } else {
            for (int i = lane; i < n; i += 64)
                sc += resid2(c[0], c[1], c[2], c[3], xs[i] - a.cx, ys[i] - a.cy, xd[i] - a.cx, yd[i] - a.cy) <= a.tau2;
        }
        sc = vs::wave_sum_i(sc);
        if (sc > best) {
            best = sc;
            best_h = h;
            for (int k = 0; k < 6; ++k) bm[k] = c[k];
        }
    }
}

__device__ __forceinline__ int model_of(int mode, int mi)
{
    const bool hybrid = mode == VS_HYBRID || mode == VS_HYBRID3;
    return !hybrid ? mode : mi == 0 ? VS_RIGID : mi == 1 ? VS_SIMILARITY : VS_AFFINE;
}

__host__ __device__ __forceinline__ int models_in(int mode) { return mode == VS_HYBRID3 ? 3 : mode == VS_HYBRID ? 2 : 1; }

// Point records of one fitted item: its slots, pair index and RANSAC stream.
struct FitItem {
    const float* src;
    const float* dst;
    const uint8_t* valid;
    int64_t pair;
    uint64_t seed;
    int64_t stream_id;
};

// item i of a strided call: pair pair_index0 + i, records at i * capacity
struct Strided {
    const float* src;
    const float* dst;
    const uint8_t* valid;
    int capacity;
    int64_t pair_index0;
    double* params;
    double* affine6;
    vs_fit_info* info;
    uint8_t* inliers;
    __device__ __forceinline__ bool at(int i, const FitArgs& a, FitItem& it) const
    {
        const int64_t k = (int64_t)i * capacity;
        it.src = src + 2 * k;
        it.dst = dst + 2 * k;
        it.valid = valid + k;
        it.pair = pair_index0 + i;
        it.seed = a.seed;
        it.stream_id = a.stream_id;
        return true;
    }
    __device__ __forceinline__ double* params_of(int i) const { return params + 4 * (int64_t)i; }
    __device__ __forceinline__ double* affine6_of(int i) const { return affine6 ? affine6 + 6 * (int64_t)i : nullptr; }
    __device__ __forceinline__ vs_fit_info* info_of(int i) const { return info + i; }
    __device__ __forceinline__ uint8_t* inliers_of(int i) const { return inliers ? inliers + (int64_t)i * capacity : nullptr; }
};

// item i of a batched step: pair j - 1 of its stream (none at j = 0), the points tracked from frame
// j - 1 (record [(j - 1) & 1]) to the tracker's outputs, the stream's own RANSAC seed and stream id
struct Step {
    vs::StepView v;
    __device__ __forceinline__ bool at(int i, const FitArgs&, FitItem& it) const
    {
        const vs::StepStream& d = v.s(i);
        const int64_t j = d.next_frame;
        if (j == 0) return false;
        const int prv = (int)((j - 1) & 1);
        it.src = d.pts + (int64_t)prv * v.capacity * 2;
        it.dst = d.dst;
        it.valid = d.status;
        it.pair = j - 1;
        it.seed = d.seed;
        it.stream_id = d.stream_id;
        return true;
    }
    __device__ __forceinline__ double* params_of(int i) const { return v.s(i).pair_params; }
    __device__ __forceinline__ double* affine6_of(int i) const { return v.s(i).affine6; }
    __device__ __forceinline__ vs_fit_info* info_of(int i) const { return v.s(i).info; }
    __device__ __forceinline__ uint8_t* inliers_of(int i) const { return v.s(i).inliers; }
};

// Kernel 1a (fit_hyp): workgroup (pair, s) of `split` per pair scores the hypotheses h = s, s + split,
// ... of every requested model (wave w takes h = s + split (w + 4k)) and records its best in the
// pair's workspace record. Splitting a pair's hypotheses over several workgroups shortens the
// dependent FP64 chains when there are few pairs.
template <class IO>
__global__ __launch_bounds__(NT, 3) void fit_hyp_kernel(IO io, int capacity, FitArgs a, int split, uint8_t* ws)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char pair_lds[];
    const int capA = lds_cap(capacity);
    float* xs = reinterpret_cast<float*>(pair_lds);
    float* ys = xs + capA;
    float* xd = ys + capA;
    float* yd = xd + capA;
    __shared__ int32_t red4[4];
    __shared__ int32_t w_score[4], w_h[4];
    __shared__ double w_model[4][6];
    const int item = blockIdx.x / split, sp = blockIdx.x - item * split;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    FitItem it;
    if (!io.at(item, a, it)) return;
    a.seed = it.seed;
    a.stream_id = it.stream_id;
    const int64_t pair = it.pair;
    HypRec* hyp = reinterpret_cast<HypRec*>(ws + item * rec_bytes(capacity) + hyp_offset(capacity));
    const int n = compact_valid(it.src, it.dst, it.valid, 0, capacity, xs, ys, xd, yd, nullptr, red4);
    const int nm = models_in(a.model);
    for (int mi = 0; mi < nm; ++mi) {
        const int model = model_of(a.model, mi);
        int best = -1, best_h = -1;
        double bm[6];
        const bool run = !(n < a.min_valid || n < 2) && a.iters > 0 && (model != VS_AFFINE || n >= 3);
        if (run) ransac_wave(model, xs, ys, xd, yd, n, a, pair, sp + split * wv, 4 * split, best, best_h, bm);
        if (lane == 0) {
            w_score[wv] = best;
            w_h[wv] = best_h;
            for (int k = 0; k < 6; ++k) w_model[wv][k] = run ? bm[k] : 0.0;
        }
        __syncthreads();
        if (t == 0) {
            int bw = -1;
            for (int w = 0; w < 4; ++w) {
                if (w_h[w] < 0) continue;
                if (bw < 0 || w_score[w] > w_score[bw] || (w_score[w] == w_score[bw] && w_h[w] < w_h[bw])) bw = w;
            }
            HypRec& r = hyp[sp * N_SLOTS + slot_of_model(model)];
            r.score = bw < 0 ? -1 : w_score[bw];
            r.h = bw < 0 ? -1 : w_h[bw];
            for (int k = 0; k < 6; ++k) r.p[k] = bw < 0 ? 0.0 : w_model[bw][k];
            r.pad = 0.0;
        }
        __syncthreads();
    }
}

template <class IO>
__global__ __launch_bounds__(NT, 3) void fit_pair_kernel(IO io, int capacity, FitArgs a, int split, uint8_t* ws)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char pair_lds[];
    const int capA = lds_cap(capacity);
    float* xs = reinterpret_cast<float*>(pair_lds);
    float* ys = xs + capA;
    float* xd = ys + capA;
    float* yd = xd + capA;
    uint16_t* slot_of = reinterpret_cast<uint16_t*>(yd + capA);
    uint8_t* inl = reinterpret_cast<uint8_t*>(slot_of + capA);
    __shared__ double red[8 * 4];
    __shared__ int32_t red4[4];
    __shared__ double w_model[1][6];
    __shared__ double s_out[6], s_tmp[4];
    __shared__ int s_best_h, s_ninl, s_flag;

    // one workgroup per (pair, model): the hybrid's candidates are fitted side by side
    const int n_models = models_in(a.model);
    const int item = blockIdx.x / n_models, mi = blockIdx.x - item * n_models, t = threadIdx.x;
    FitItem it;
    if (!io.at(item, a, it)) return;
    PairRec* rec = reinterpret_cast<PairRec*>(ws + item * rec_bytes(capacity));
    uint8_t* masks = ws + item * rec_bytes(capacity) + 256;
    const int model = model_of(a.model, mi);

    const int n = compact_valid(it.src, it.dst, it.valid, 0, capacity, xs, ys, xd, yd, slot_of, red4);
    const HypRec* hyp = reinterpret_cast<const HypRec*>(ws + item * rec_bytes(capacity) + hyp_offset(capacity));
    uint8_t* mk = masks + slot_of_model(model) * cap_aligned(capacity);
    for (int k = t; k < cap_aligned(capacity); k += NT) mk[k] = 0;
    __syncthreads();
    if (t == 0 && mi == 0) {
        rec->n_valid = n;
        rec->skipped = (n < a.min_valid || n < 2) ? 1 : 0;
    }
    if (n < a.min_valid || n < 2) return;

    {
        const bool affine = model == VS_AFFINE;
        bool have = false;
        if (a.iters > 0 && (!affine || n >= 3)) {
            // the best of the hypothesis workgroups' bests: most inliers, then the smallest h. Wave 0
            // reads one record per lane and takes the maximum of the key (score + 1, ~h); records
            // without a hypothesis (h < 0) have key 0. Hypothesis indices are distinct, so the
            // maximum is unique.
            if (t < 64) {
                uint64_t key = 0;
                if (t < split) {
                    const HypRec& r = hyp[t * N_SLOTS + slot_of_model(model)];
                    if (r.h >= 0)
                        key = ((uint64_t)(uint32_t)(r.score + 1) << 32) | (uint64_t)(0xffffffffu - (uint32_t)r.h);
                }
                uint64_t m = key;
#pragma unroll
                for (int d = 32; d >= 1; d >>= 1) {
                    const uint64_t o = __shfl_xor(m, d, 64);
                    m = o > m ? o : m;
                }
                if (m != 0 && key == m)
                    for (int k = 0; k < 6; ++k) w_model[0][k] = hyp[t * N_SLOTS + slot_of_model(model)].p[k];
                if (t == 0) s_best_h = m == 0 ? -1 : 0;
            }
            __syncthreads();
            const int bw = s_best_h;
            if (bw >= 0) {
                const double* c = w_model[bw];
                int m = 0;
                for (int i = t; i < n; i += NT) {
                    const double x = xs[i] - a.cx, y = ys[i] - a.cy, u = xd[i] - a.cx, w = yd[i] - a.cy;
                    const uint8_t f = (affine ? aff_resid2(c, x, y, u, w) : resid2(c[0], c[1], c[2], c[3], x, y, u, w)) <=
                                      a.tau2;
                    inl[i] = f;
                    m += f;
                }
                m = block_sum_i(m, red4);
                if (t == 0) s_ninl = m;
                __syncthreads();
                have = s_ninl >= (affine ? 3 : 2);
            }
        }
        if (!have) {
            for (int i = t; i < n; i += NT) inl[i] = 1;
            if (t == 0) s_ninl = n;
            __syncthreads();
        }
        if (affine)
            ls_affine(xs, ys, xd, yd, a.cx, a.cy, inl, n, red, s_out, s_tmp, &s_flag);
        else
            ls_refit(model, xs, ys, xd, yd, a.cx, a.cy, inl, n, red, s_out);
        // RMS residual of the refitted model over all valid points
        double e[1] = {0.0};
        double q[6];
        for (int k = 0; k < 6; ++k) q[k] = s_out[k];
        for (int i = t; i < n; i += NT) {
            const double x = xs[i] - a.cx, y = ys[i] - a.cy, u = xd[i] - a.cx, w = yd[i] - a.cy;
            e[0] += affine ? aff_resid2(q, x, y, u, w) : resid2(q[0], q[1], q[2], q[3], x, y, u, w);
        }
        block_sum<1>(e, red);
        const int slot = slot_of_model(model);
        if (t == 0) {
            ModelFit& mf = rec->m[slot];
            for (int k = 0; k < 6; ++k) mf.p[k] = (affine || k < 4) ? s_out[k] : 0.0;
            mf.err = sqrt(e[0] / n);
            mf.n_inl = s_ninl;
        }
        for (int i = t; i < n; i += NT) mk[slot_of[i]] = inl[i];
    }
}

// Runs the dwell-block state machine over the pairs of the call and records each pair's choice in
// its workspace record. It is evaluated block-parallel, with the same result as walking the pairs in
// order: a block's decision pair is its first non-skipped pair in the call (none if the incoming
// state already decided that block); the model in force before it is the last decision of an earlier
// block (or the incoming model); pairs from the decision on use the block's decision. Blocks are
// taken in chunks of NB: one thread per block finds the decision, one thread carries the model
// across the chunk's blocks, then every pair of the chunk writes its choice.
constexpr int NB = 1024;

__device__ __forceinline__ int decide(int model_mode, double er, double es, double ea)
{
    int m = (er < es) ? VS_RIGID : VS_SIMILARITY;
    if (model_mode == VS_HYBRID3 && ea < (m == VS_RIGID ? er : es)) m = VS_AFFINE;
    return m;
}

__global__ __launch_bounds__(NT) void fit_resolve_kernel(int n, int capacity, FitArgs a, int64_t pair_index0,
                                                         vs_fit_state* state, uint8_t* ws)
{
    __shared__ int32_t dec_pair[NB];
    __shared__ int8_t dec_model[NB], model_before[NB];
    __shared__ int32_t s_carry;
    const int t = threadIdx.x;
    const vs_fit_state st_in = *state;
    const bool hybrid = a.model == VS_HYBRID || a.model == VS_HYBRID3;
    const int64_t dw = a.dwell > 0 ? a.dwell : 1;
    const int64_t blk_first = pair_index0 / dw, blk_last = (pair_index0 + n - 1) / dw;
    const bool first_done = st_in.block == blk_first && st_in.decided;   // block decided by an earlier call
    if (t == 0) s_carry = st_in.model;
    __syncthreads();
    for (int64_t b0 = blk_first; b0 <= blk_last; b0 += NB) {
        const int nb = (int)min((int64_t)NB, blk_last - b0 + 1);
        // 1. decision pair and model of every block of the chunk
        for (int k = t; k < nb; k += NT) {
            const int64_t b = b0 + k;
            const int64_t p0 = max(b * dw, pair_index0) - pair_index0;
            const int64_t p1 = min((b + 1) * dw, pair_index0 + n) - pair_index0;
            int dp = -1, dm = -1;
            if (hybrid && !(b == blk_first && first_done)) {
                for (int64_t i = p0; i < p1; ++i) {
                    const PairRec* rec = reinterpret_cast<const PairRec*>(ws + i * rec_bytes(capacity));
                    if (!rec->skipped) {
                        dp = (int)i;
                        dm = decide(a.model, rec->m[0].err, rec->m[1].err, rec->m[2].err);
                        break;
                    }
                }
            }
            dec_pair[k] = dp;
            dec_model[k] = (int8_t)dm;
        }
        __syncthreads();
        // 2. model in force at the start of every block
        if (t == 0) {
            int carry = s_carry;
            for (int k = 0; k < nb; ++k) {
                model_before[k] = (int8_t)carry;
                if (dec_model[k] >= 0) carry = dec_model[k];
            }
            s_carry = carry;
        }
        __syncthreads();
        // 3. every pair of the chunk's blocks
        const int64_t q0 = max(b0 * dw, pair_index0) - pair_index0;
        const int64_t q1 = min((b0 + nb) * dw, pair_index0 + n) - pair_index0;
        for (int64_t i = q0 + t; i < q1; i += NT) {
            PairRec* rec = reinterpret_cast<PairRec*>(ws + i * rec_bytes(capacity));
            const int k = (int)((pair_index0 + i) / dw - b0);
            int m = a.model, dh = 0;
            if (hybrid) {
                const int dp = dec_pair[k];
                m = (dp >= 0 && i >= dp) ? dec_model[k] : model_before[k];
                dh = dp == (int)i;
            }
            rec->pad[0] = rec->skipped ? -1 - m : m;   // a skipped pair is the identity under the reported model
            rec->pad[1] = dh;
        }
        __syncthreads();
    }
    if (t == 0) {
        vs_fit_state st = st_in;
        if (st.block != blk_last) {
            st.block = blk_last;
            st.decided = 0;
        }
        if (hybrid) {
            st.model = s_carry;
            // the last block is decided if its decision pair lies in this call (or an earlier call made it)
            const int64_t k_last = (blk_last - blk_first) % NB;
            if (dec_pair[k_last] >= 0) st.decided = 1;
        }
        *state = st;
    }
}

// One workgroup per pair: writes the chosen model's parameters (an affine as its nearest
// similarity, a = (a11 + a22) / 2, b = (a21 - a12) / 2), the 2x3 matrices (optional), info record
// and inlier flags.
template <class IO>
__global__ __launch_bounds__(NT) void fit_emit_kernel(int capacity, int32_t model_mode, const uint8_t* ws, IO io,
                                                      FitArgs a)
{
    const int i = blockIdx.x, t = threadIdx.x;
    FitItem it;
    if (!io.at(i, a, it)) return;
    double* __restrict__ affine6 = io.affine6_of(i);
    uint8_t* __restrict__ inliers = io.inliers_of(i);
    const PairRec* rec = reinterpret_cast<const PairRec*>(ws + i * rec_bytes(capacity));
    const int ch = rec->pad[0];
    if (t == 0) {
        vs_fit_info f;
        f.n_valid = rec->n_valid;
        f.skipped = rec->skipped;
        f.decided_here = rec->pad[1];
        f.pad = 0;
        f.err_rigid = __longlong_as_double(0x7ff8000000000000ll);
        f.err_sim = f.err_rigid;
        f.err_affine = f.err_rigid;
        double* po = io.params_of(i);
        double m6[6] = {1.0, 0.0, 0.0, 0.0, 1.0, 0.0};
        if (ch < 0) {
            f.model = -1 - ch;
            f.n_inliers = 0;
            po[0] = 1.0; po[1] = 0.0; po[2] = 0.0; po[3] = 0.0;
        } else {
            const ModelFit& mf = rec->m[slot_of_model(ch)];
            f.model = ch;
            f.n_inliers = mf.n_inl;
            if (ch == VS_AFFINE) {
                for (int k = 0; k < 6; ++k) m6[k] = mf.p[k];
                po[0] = (m6[0] + m6[4]) * 0.5;
                po[1] = (m6[3] - m6[1]) * 0.5;
                po[2] = m6[2];
                po[3] = m6[5];
            } else {
                for (int k = 0; k < 4; ++k) po[k] = mf.p[k];
                m6[0] = mf.p[0]; m6[1] = -mf.p[1]; m6[2] = mf.p[2];
                m6[3] = mf.p[1]; m6[4] = mf.p[0];  m6[5] = mf.p[3];
            }
            if (f.decided_here) {
                f.err_rigid = rec->m[0].err;
                f.err_sim = rec->m[1].err;
                if (model_mode == VS_HYBRID3) f.err_affine = rec->m[2].err;
            }
        }
        if (affine6)
            for (int k = 0; k < 6; ++k) affine6[k] = m6[k];
        *io.info_of(i) = f;
    }
    if (inliers) {
        const uint8_t* mk = ws + i * rec_bytes(capacity) + 256 + (ch < 0 ? 0 : slot_of_model(ch)) * cap_aligned(capacity);
        for (int k = t; k < capacity; k += NT) inliers[k] = ch < 0 ? 0 : mk[k];
    }
}

// The dwell-block state machine for a batched step: item i fits one pair (j - 1) of its own stream,
// so each item is resolved alone by one thread, exactly as fit_resolve_kernel resolves a call of one
// pair: a hybrid block is decided at its first non-skipped pair (unless the state already decided
// it); the model in force is carried otherwise.
__global__ void fit_resolve_step_kernel(int n, int capacity, FitArgs a, vs::StepView v, uint8_t* ws)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    vs::StepStream& d = v.s(i);
    if (d.next_frame == 0) return;
    const int64_t pair = d.next_frame - 1;
    PairRec* rec = reinterpret_cast<PairRec*>(ws + i * rec_bytes(capacity));
    const bool hybrid = a.model == VS_HYBRID || a.model == VS_HYBRID3;
    const int64_t dw = a.dwell > 0 ? a.dwell : 1;
    const int64_t blk = pair / dw;
    vs_fit_state st = *d.fit_state;
    const bool done = st.block == blk && st.decided;
    int m = a.model, dh = 0;
    if (hybrid) {
        m = st.model;
        if (!done && !rec->skipped) {
            m = decide(a.model, rec->m[0].err, rec->m[1].err, rec->m[2].err);
            dh = 1;
        }
    }
    rec->pad[0] = rec->skipped ? -1 - m : m;   // a skipped pair is the identity under the reported model
    rec->pad[1] = dh;
    if (st.block != blk) {
        st.block = blk;
        st.decided = 0;
    }
    if (hybrid) {
        st.model = m;
        if (dh) st.decided = 1;
    }
    *d.fit_state = st;
}

__global__ void fit_state_init_kernel(vs_fit_state* s)
{
    s->block = -1;
    s->model = VS_SIMILARITY;
    s->decided = 0;
}

}  // namespace

extern "C" size_t vs_fit_workspace(int32_t n, int32_t capacity)
{
    if (n <= 0 || capacity <= 0) return 0;
    return (size_t)rec_bytes(capacity) * (size_t)n;
}

extern "C" int vs_fit_state_init(vs_fit_state* state, void* stream)
{
    if (!state) return vs::set_error(VS_ERR_INVALID, "vs_fit_state_init: null state");
    fit_state_init_kernel<<<1, 1, 0, vs::as_stream(stream)>>>(state);
    return vs::check_launch("vs_fit_state_init");
}

namespace {

// Validates the arguments shared by both fit entry points; on success fills *a.
int check_fit_args(const char* who, const float* src, const float* dst, const uint8_t* valid, int32_t capacity,
                   int32_t n, const vs_fit_params* p, int64_t pair_index0, const vs_fit_state* state,
                   const double* params, const vs_fit_info* info, FitArgs* a)
{
    if (!p) return vs::set_error(VS_ERR_INVALID, "%s: null params", who);
    if (n < 0 || capacity <= 0) return vs::set_error(VS_ERR_INVALID, "%s: bad count or capacity", who);
    if (n == 0) return VS_OK;
    if (!src || !dst || !valid || !state || !params || !info)
        return vs::set_error(VS_ERR_INVALID, "%s: null argument", who);
    if (capacity > VS_MAX_CORNERS) return vs::set_error(VS_ERR_UNSUPPORTED, "%s: capacity > %d", who, VS_MAX_CORNERS);
    const bool with_affine = p->model == VS_AFFINE || p->model == VS_HYBRID3;
    if (p->model < VS_RIGID || p->model > VS_HYBRID3 || p->ransac_iters < 0 ||
        p->ransac_iters > (with_affine ? 8191 : 32767) || !(p->inlier_thresh >= 0.0) || p->dwell < 1 || pair_index0 < 0)
        return vs::set_error(VS_ERR_INVALID, "%s: bad parameters", who);
    if (n > 65535) return vs::set_error(VS_ERR_INVALID, "%s: more than 65535 pairs", who);
    a->model = p->model;
    a->iters = p->ransac_iters;
    a->tau2 = p->inlier_thresh * p->inlier_thresh;
    a->seed = p->seed;
    a->stream_id = p->stream_id;
    a->min_valid = p->min_valid;
    a->dwell = p->dwell;
    a->cx = p->cx;
    a->cy = p->cy;
    return VS_OK;
}

// Enqueues the four fit kernels over a workspace of at least vs_fit_workspace(n, capacity) bytes
// (a device address, 256-byte aligned; its contents on entry do not matter: every byte the kernels
// read is written earlier in the same call).
int launch_fit(const char* who, const float* src, const float* dst, const uint8_t* valid, int32_t capacity, int32_t n,
               const FitArgs& a, int64_t pair_index0, vs_fit_state* state, double* params, double* affine6,
               vs_fit_info* info, uint8_t* inliers, uint8_t* w8, hipStream_t s)
{
    const size_t lds = pair_lds_bytes(capacity);
    if (lds > 65536) {
        // capacities above ~3400 points need more than the default 64 KiB of dynamic LDS
        hipError_t he = hipFuncSetAttribute(reinterpret_cast<const void*>(&fit_pair_kernel<Strided>),
                                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (he == hipSuccess)
            he = hipFuncSetAttribute(reinterpret_cast<const void*>(&fit_hyp_kernel<Strided>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (he != hipSuccess) return vs::set_error(VS_ERR_HIP, "%s: %s", who, hipGetErrorString(he));
    }
    // spread each pair's hypotheses over workgroups until about fit_groups_in_flight (2048 by default)
    // are in flight (up to MAX_SPLIT per pair): the scoring loops are chains of dependent FP64
    // operations, hidden only by other waves
    const int target = vs::fit_groups_in_flight();
    const int split = a.iters > 0 ? std::min(std::max((target + n - 1) / n, 1), MAX_SPLIT) : 1;
    const Strided io{src, dst, valid, capacity, pair_index0, params, affine6, info, inliers};
    fit_hyp_kernel<<<n * split, NT, lds, s>>>(io, capacity, a, split, w8);
    int e = vs::check_launch(who);
    if (e) return e;
    fit_pair_kernel<<<n * models_in(a.model), NT, lds, s>>>(io, capacity, a, split, w8);
    if ((e = vs::check_launch(who))) return e;
    fit_resolve_kernel<<<1, NT, 0, s>>>(n, capacity, a, pair_index0, state, w8);
    if ((e = vs::check_launch(who))) return e;
    fit_emit_kernel<<<n, NT, 0, s>>>(capacity, a.model, w8, io, a);
    return vs::check_launch(who);
}

// the fit of every item of a batched step with j > 0
int launch_fit_step(const vs::StepView& v, int n, const FitArgs& a, uint8_t* w8, hipStream_t s)
{
    const char* who = "vs_batch_push(fit)";
    const int capacity = v.capacity;
    const size_t lds = pair_lds_bytes(capacity);
    if (lds > 65536) {
        hipError_t he = hipFuncSetAttribute(reinterpret_cast<const void*>(&fit_pair_kernel<Step>),
                                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (he == hipSuccess)
            he = hipFuncSetAttribute(reinterpret_cast<const void*>(&fit_hyp_kernel<Step>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (he != hipSuccess) return vs::set_error(VS_ERR_HIP, "%s: %s", who, hipGetErrorString(he));
    }
    const Step io{v};
    const int target = vs::fit_groups_in_flight();
    const int split = a.iters > 0 ? std::min(std::max((target + n - 1) / n, 1), MAX_SPLIT) : 1;
    fit_hyp_kernel<<<n * split, NT, lds, s>>>(io, capacity, a, split, w8);
    int e = vs::check_launch(who);
    if (e) return e;
    fit_pair_kernel<<<n * models_in(a.model), NT, lds, s>>>(io, capacity, a, split, w8);
    if ((e = vs::check_launch(who))) return e;
    fit_resolve_step_kernel<<<(n + 63) / 64, 64, 0, s>>>(n, capacity, a, v, w8);
    if ((e = vs::check_launch(who))) return e;
    fit_emit_kernel<<<n, NT, 0, s>>>(capacity, a.model, w8, io, a);
    return vs::check_launch(who);
}

// Scratch of vs_fit_motion_noalloc: a file-scope device array, one copy per GPU, held until the
// process ends. Host code never passes `scratch` itself to a kernel (on the host the name is only a
// stand-in for the symbol): it looks up each device's address once, with that device current, and
// passes that address.
static __device__ __align__(256) uint8_t scratch[VS_FIT_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

int scratch_address(const char* who, hipStream_t s, uint8_t** out)
{
    int dev = -1;
    hipError_t he = hipGetDevice(&dev);
    if (he != hipSuccess) return vs::set_error(VS_ERR_HIP, "%s: hipGetDevice: %s", who, hipGetErrorString(he));
    if (dev < 0 || dev >= MAX_DEVICES) return vs::set_error(VS_ERR_UNSUPPORTED, "%s: device %d", who, dev);
    if (s) {
        // the scratch must live on the device the work runs on
        hipDevice_t sd = -1;
        he = hipStreamGetDevice(s, &sd);
        if (he != hipSuccess)
            return vs::set_error(VS_ERR_HIP, "%s: hipStreamGetDevice: %s", who, hipGetErrorString(he));
        if (sd != dev) return vs::set_error(VS_ERR_INVALID, "%s: stream of device %d, device %d current", who, sd, dev);
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        he = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (he != hipSuccess || !p)
            return vs::set_error(VS_ERR_HIP, "%s: hipGetSymbolAddress: %s", who, hipGetErrorString(he));
        g_scratch_ptr[dev] = p;
    }
    *out = static_cast<uint8_t*>(g_scratch_ptr[dev]);
    return VS_OK;
}

}  // namespace

extern "C" int vs_fit_motion(const float* src, const float* dst, const uint8_t* valid, int32_t capacity, int32_t n,
                             const vs_fit_params* p, int64_t pair_index0, vs_fit_state* state, double* params,
                             double* affine6, vs_fit_info* info, uint8_t* inliers, void* workspace, size_t ws_bytes,
                             void* stream)
{
    FitArgs a;
    int e = check_fit_args("vs_fit_motion", src, dst, valid, capacity, n, p, pair_index0, state, params, info, &a);
    if (e || n == 0) return e;
    if (!workspace) return vs::set_error(VS_ERR_INVALID, "vs_fit_motion: null argument");
    const size_t need = vs_fit_workspace(n, capacity);
    if (ws_bytes < need) return vs::set_error(VS_ERR_WORKSPACE, "vs_fit_motion: workspace %zu < %zu", ws_bytes, need);
    if (reinterpret_cast<uintptr_t>(workspace) & 255)
        return vs::set_error(VS_ERR_INVALID, "vs_fit_motion: workspace must be 256-byte aligned");
    return launch_fit("vs_fit_motion", src, dst, valid, capacity, n, a, pair_index0, state, params, affine6, info,
                      inliers, static_cast<uint8_t*>(workspace), vs::as_stream(stream));
}

extern "C" int32_t vs_fit_noalloc_max_pairs(int32_t capacity)
{
    if (capacity <= 0 || capacity > VS_MAX_CORNERS) return 0;
    return (int32_t)std::min<int64_t>(65535, (int64_t)VS_FIT_NOALLOC_SCRATCH_BYTES / rec_bytes(capacity));
}

extern "C" int vs_fit_motion_noalloc(const float* src, const float* dst, const uint8_t* valid, int32_t capacity,
                                     int32_t n, const vs_fit_params* p, int64_t pair_index0, vs_fit_state* state,
                                     double* params, double* affine6, vs_fit_info* info, uint8_t* inliers, void* stream)
{
    const char* who = "vs_fit_motion_noalloc";
    FitArgs a;
    int e = check_fit_args(who, src, dst, valid, capacity, n, p, pair_index0, state, params, info, &a);
    if (e || n == 0) return e;
    const int32_t max_n = vs_fit_noalloc_max_pairs(capacity);
    if (n > max_n)
        return vs::set_error(VS_ERR_WORKSPACE, "%s: %d pairs of capacity %d need %zu bytes of scratch; at most %d pairs "
                             "fit its %d bytes", who, n, capacity, vs_fit_workspace(n, capacity), max_n,
                             (int)VS_FIT_NOALLOC_SCRATCH_BYTES);
    hipStream_t s = vs::as_stream(stream);
    uint8_t* w8 = nullptr;
    if ((e = scratch_address(who, s, &w8))) return e;
    return launch_fit(who, src, dst, valid, capacity, n, a, pair_index0, state, params, affine6, info, inliers, w8, s);
}

extern "C" int vs_fit_similarity(const float* src, const float* dst, const uint8_t* valid, int32_t capacity, int32_t n,
                                 const vs_fit_params* p, int64_t pair_index0, vs_fit_state* state, double* params,
                                 vs_fit_info* info, uint8_t* inliers, void* workspace, size_t ws_bytes, void* stream)
{
    return vs_fit_motion(src, dst, valid, capacity, n, p, pair_index0, state, params, nullptr, info, inliers, workspace,
                         ws_bytes, stream);
}

namespace vs {

size_t step_fit_workspace(int n, int capacity) { return vs_fit_workspace(n, capacity); }

int step_fit(const StepView& v, int n, const vs_fit_params& p, uint8_t* ws, hipStream_t s)
{
    if (n <= 0) return VS_OK;
    FitArgs a;
    // the point pointers are only checked for null: the step's come from the descriptors
    const float one = 0.f;
    const uint8_t flag = 0;
    const vs_fit_state st{};
    const double prm = 0.0;
    const vs_fit_info inf{};
    const int e = check_fit_args("vs_batch_push(fit)", &one, &one, &flag, v.capacity, n, &p, 0, &st, &prm, &inf, &a);
    if (e) return e;
    return launch_fit_step(v, n, a, ws, s);
}

}  // namespace vs
