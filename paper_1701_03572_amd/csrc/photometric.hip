// Photometric check and refinement of fitted pair similarities (an extension: the brightness
// constancy of Eq. 3 applied to the whole frame under the similarity of Eq. 7).
//
// The sampler S(F, p) is the bilinear interpolant of F extended by edge replication; its gradient
// is the derivative of the bilinear piece in cell floor(p). The transform is
// T(x) = x + [[a, -b], [b, a]] (x - c) / rho + t, theta = (a, b, tx, ty). Per pixel of the rectangle
// Omega the residual is r = S(F1, T(x)) - F0(x) and its Jacobian row J = grad S . dT/dtheta.
//
// Arithmetic is binary64 throughout: vector FP64 issues at the rate of unpacked FP32 on this
// hardware, and every pass is small next to the tracker.
//
// photo_sums_kernel: a 256-thread workgroup covers a 256 x 32 tile of Omega (4 x 8 pixels per thread),
// reads its taps from LDS copies of the tile and of the tile's source box in the next frame, and
// accumulates the loss, J^T J (upper triangle) and J^T r; the per-thread sums are reduced over the
// workgroup in a fixed order and stored as the tile's 19 partial sums in the workspace (the gradient
// as twice the J^T r sums, which it equals exactly). photo_reduce_kernel: one workgroup per pair adds its tiles' partials, again in a fixed
// order (tile t goes to thread t mod 256, the threads' totals through a wave butterfly and the four
// wave totals in sequence), so every sum is reproducible bit for bit from run to run.
// photo_feature_kernel: one wave per point; the window's samples are spread over the lanes.
// Refinement: per step, one sums pass at the candidate parameters and one small kernel per pair that
// accepts the candidate if its loss is lower, solves (J^T J) delta = -J^T r by Cholesky at the
// accepted parameters and forms the next candidate. A pair stops at its first rejected step.
#include "vs_common.hpp"

namespace {

constexpr int NACC = 19;              // loss, grad[4], upper(J^T J)[10], J^T r[4]
constexpr int TW = 256, RPT = 8, TH = 4 * RPT;

struct PhotoState {
    double theta[4];                  // accepted parameters
    double cand[4];                   // candidate of the running step
    double cur[NACC];                 // sums at theta
    double nxt[NACC];                 // sums at cand
    double loss0;
    int32_t stopped;
    int32_t accepted;
};

struct Frame {
    const uint8_t* p;
    int w, h, pitch;
};

__device__ __forceinline__ double px(const Frame& f, int x, int y)
{
    x = x < 0 ? 0 : (x > f.w - 1 ? f.w - 1 : x);
    y = y < 0 ? 0 : (y > f.h - 1 ? f.h - 1 : y);
    return (double)f.p[(int64_t)y * f.pitch + x];
}

// bilinear value and gradient at (x, y)
__device__ __forceinline__ void sample_grad(const Frame& f, double x, double y, double& v, double& gx, double& gy)
{
    const double fx = floor(x), fy = floor(y);
    const double a = x - fx, b = y - fy;
    const int x0 = (int)fx, y0 = (int)fy;
    const double p00 = px(f, x0, y0), p10 = px(f, x0 + 1, y0), p01 = px(f, x0, y0 + 1), p11 = px(f, x0 + 1, y0 + 1);
    const double top = fma(a, p10 - p00, p00), bot = fma(a, p11 - p01, p01);
    v = fma(b, bot - top, top);
    gx = fma(b, (p11 - p01) - (p10 - p00), p10 - p00);
    gy = fma(a, (p11 - p10) - (p01 - p00), p01 - p00);
}

__device__ __forceinline__ double sample(const Frame& f, double x, double y)
{
    const double fx = floor(x), fy = floor(y);
    const double a = x - fx, b = y - fy;
    const int x0 = (int)fx, y0 = (int)fy;
    const double p00 = px(f, x0, y0), p10 = px(f, x0 + 1, y0), p01 = px(f, x0, y0 + 1), p11 = px(f, x0 + 1, y0 + 1);
    const double top = fma(a, p10 - p00, p00), bot = fma(a, p11 - p01, p01);
    return fma(b, bot - top, top);
}

// Staged source boxes: a tile's pixels map (affinely) into a box of the next frame, which is staged in
// LDS with 16-byte loads, rows and columns clamped to the frame (the sampler's edge replication), and
// so is the tile of the previous frame; every tap is then an LDS byte read. Boxes larger than the
// buffer take the direct path (per-tap global loads).
constexpr int SLP = 288;                 // LDS row pitch of the staged blocks (18 chunks of 16 bytes)
constexpr int SNCH = SLP / 16;
constexpr int SMAXR = 79;                // staged next-frame rows at most (the LDS of 5 workgroups per CU)
constexpr double SBIG = 1048576.0;       // boxes beyond +-2^20 take the direct path
constexpr uint32_t RSRC_WORD3 = 0x00020000;   // raw (untyped) buffer access on gfx9-family parts

// the position in the next frame of pixel (x, y), dx = (x - cx) / rho and dy = (y - cy) / rho
__device__ __forceinline__ void map_px(int x, double dx, int y, double dy, double t0, double t1, double t2, double t3,
                                       double& px_, double& py_)
{
    px_ = (double)x + t0 * dx - t1 * dy + t2;
    py_ = (double)y + t1 * dx + t0 * dy + t3;
}

// Adds one pixel's residual (and with need_grad its Jacobian row's products) to the thread's sums.
// The gradient slots 1..4 are left alone: the gradient's sum is 2 J^T r exactly (doubling is exact,
// so fma(2 r, J, 2 s) = 2 fma(r, J, s) at every step, and so for every sum of such terms in a fixed
// order), and the tile's gradient is written as twice its J^T r.
__device__ __forceinline__ void accumulate(double res, double gx, double gy, double dx, double dy, int need_grad,
                                           double (&s)[NACC])
{
    s[0] = fma(res, res, s[0]);
    if (need_grad) {
        const double J[4] = {gx * dx + gy * dy, gy * dx - gx * dy, gx, gy};
        int t = 5;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            s[15 + i] = fma(J[i], res, s[15 + i]);
#pragma unroll
            for (int j = i; j < 4; ++j) {
                s[t] = fma(J[i], J[j], s[t]);
                ++t;
            }
        }
    }
}

// Stages rows r0 .. r0 + nr - 1 (each clamped to the frame) and the 16-byte chunks starting at column
// c0 (c0 a multiple of 16; columns clamped to the frame) of F into buf (row r at r * SLP).
__device__ __forceinline__ void stage_block(const Frame& F, bool vec_ok, int r0, int nr, int c0, int nch, uint8_t* buf)
{
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t*>(F.p), (short)0,
                                                                        F.pitch * F.h, RSRC_WORD3);
    using V4 = __attribute__((ext_vector_type(4))) unsigned int;
    for (int k = threadIdx.x; k < nr * nch; k += blockDim.x) {
        const int r = k / nch, c = k - r * nch;
        const int gy = vs::clampi(r0 + r, 0, F.h - 1);
        const int gx = c0 + 16 * c;
        V4 v;
        if (vec_ok && gx >= 0 && gx + 16 <= F.w) {
            v = __builtin_bit_cast(V4, __builtin_amdgcn_raw_buffer_load_b128(rs, gy * F.pitch + gx, 0, 0));
        } else {
            uint32_t wd[4] = {0u, 0u, 0u, 0u};
            for (int e = 0; e < 16; ++e) {
                const uint32_t byte = __builtin_amdgcn_raw_buffer_load_b8(rs, gy * F.pitch + vs::clampi(gx + e, 0, F.w - 1),
                                                                         0, 0);
                wd[e >> 2] |= byte << (8 * (e & 3));
            }
            v = V4{wd[0], wd[1], wd[2], wd[3]};
        }
        *reinterpret_cast<V4*>(&buf[r * SLP + 16 * c]) = v;
    }
}

// Which parameters: theta_src[item * tstride] when state == nullptr, else the state's candidate
// (pairs already stopped are skipped). The tile's sums go to part[(item * tiles + tile) * NACC + k]
// for k < 1 (loss only) or k < NACC.
__global__ __launch_bounds__(256) void photo_sums_kernel(const uint8_t* __restrict__ prev, const uint8_t* __restrict__ next,
                                                         int64_t fstride, int W, int H, int pitch, const double* theta_src,
                                                         int64_t tstride, const PhotoState* state, double cx, double cy,
                                                         double rho, int ox0, int oy0, int ox1, int oy1, int need_grad,
                                                         double* __restrict__ part, int tiles_x, int tiles_y)
{
    __shared__ double red[4][NACC];
    __shared__ __attribute__((aligned(16))) uint8_t box1[SMAXR * SLP];   // the next frame's source box
    __shared__ __attribute__((aligned(16))) uint8_t box0[TH * SLP];      // the previous frame's tile
    const int tiles = tiles_x * tiles_y;
    const int item = blockIdx.x / tiles, tile = blockIdx.x - item * tiles;
    const double* th;
    if (state) {
        if (state[item].stopped) return;
        th = state[item].cand;
    } else {
        th = theta_src + item * tstride;
    }
    double* out = part + ((int64_t)item * tiles + tile) * NACC;
    const int ty = tile / tiles_x, tx = tile - ty * tiles_x;
    const Frame F0{prev + item * fstride, W, H, pitch}, F1{next + item * fstride, W, H, pitch};
    const double t0 = th[0], t1 = th[1], t2 = th[2], t3 = th[3];
    const int xb = ox0 + tx * TW + (threadIdx.x & 63) * 4;
    const int yb = oy0 + ty * TH + (threadIdx.x >> 6) * RPT;
    double s[NACC];
#pragma unroll
    for (int k = 0; k < NACC; ++k) s[k] = 0.0;

    // the tile's pixels [X0, X1) x [Y0, Y1); their positions are monotone in x and in y (every operation
    // rounds monotonically), so the box of the four corners, widened by one pixel, holds every tap
    const int X0 = ox0 + tx * TW, X1 = min(X0 + TW, ox1), Y0 = oy0 + ty * TH, Y1 = min(Y0 + TH, oy1);
    double mnx = INFINITY, mxx = -INFINITY, mny = INFINITY, mxy = -INFINITY;
    bool finite = true;
#pragma unroll
    for (int cyi = 0; cyi < 2; ++cyi)
#pragma unroll
        for (int cxi = 0; cxi < 2; ++cxi) {
            const int x = cxi ? X1 - 1 : X0, y = cyi ? Y1 - 1 : Y0;
            double qx, qy;
            map_px(x, ((double)x - cx) / rho, y, ((double)y - cy) / rho, t0, t1, t2, t3, qx, qy);
            mnx = fmin(mnx, qx);
            mxx = fmax(mxx, qx);
            mny = fmin(mny, qy);
            mxy = fmax(mxy, qy);
            finite = finite && qx > -SBIG && qx < SBIG && qy > -SBIG && qy < SBIG;   // false for NaN
        }
    int a0 = 0, by0 = 0, nr = 0;
    // a map far from degenerate (|t0|, |t1| < rho / 2): each position moves by at least half a pixel
    // per pixel along its own axis, so the corners bound the tile
    bool staged = finite && fabs(t0) < 0.5 * rho && fabs(t1) < 0.5 * rho;
    if (staged) {
        a0 = ((int)floor(mnx) - 1) & ~15;
        by0 = (int)floor(mny) - 1;
        nr = (int)floor(mxy) + 2 - by0 + 1;
        staged = (int)floor(mxx) + 2 - a0 < SLP && nr <= SMAXR;
    }
    if (staged) {
        const int c00 = X0 & ~15;
        stage_block(F1, ((reinterpret_cast<uintptr_t>(F1.p) | (uintptr_t)pitch) & 15) == 0, by0, nr, a0, SNCH, box1);
        stage_block(F0, ((reinterpret_cast<uintptr_t>(F0.p) | (uintptr_t)pitch) & 15) == 0, Y0, Y1 - Y0, c00,
                    min(SNCH, (X1 - c00 + 15) / 16), box0);
        __syncthreads();
        double dxq[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) dxq[q] = ((double)(xb + q) - cx) / rho;
        for (int r = 0; r < RPT; ++r) {
            const int y = yb + r;
            if (y >= oy1) break;
            const double dy = ((double)y - cy) / rho;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int x = xb + q;
                if (x >= ox1) break;
                const double dx = dxq[q];
                double px_, py_;
                map_px(x, dx, y, dy, t0, t1, t2, t3, px_, py_);
                // the sampler of sample_grad, its taps read from the staged box
                const double fx = floor(px_), fy = floor(py_);
                const double a = px_ - fx, b = py_ - fy;
                const int o = ((int)fy - by0) * SLP + ((int)fx - a0);
                const double p00 = box1[o], p10 = box1[o + 1], p01 = box1[o + SLP], p11 = box1[o + SLP + 1];
                const double top = fma(a, p10 - p00, p00), bot = fma(a, p11 - p01, p01);
                const double v = fma(b, bot - top, top);
                const double gx = fma(b, (p11 - p01) - (p10 - p00), p10 - p00);
                const double gy = fma(a, (p11 - p10) - (p01 - p00), p01 - p00);
                const double res = v - (double)box0[(y - Y0) * SLP + (x - c00)];
                accumulate(res, gx, gy, dx, dy, need_grad, s);
            }
        }
    } else {
        for (int r = 0; r < RPT; ++r) {
            const int y = yb + r;
            if (y >= oy1) break;
            const double dy = ((double)y - cy) / rho;
            for (int q = 0; q < 4; ++q) {
                const int x = xb + q;
                if (x >= ox1) break;
                const double dx = ((double)x - cx) / rho;
                double px_, py_;
                map_px(x, dx, y, dy, t0, t1, t2, t3, px_, py_);
                double v, gx, gy;
                sample_grad(F1, px_, py_, v, gx, gy);
                const double res = v - (double)F0.p[(int64_t)y * pitch + x];
                accumulate(res, gx, gy, dx, dy, need_grad, s);
            }
        }
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int nk = need_grad ? NACC : 1;
#pragma unroll
    for (int k = 0; k < NACC; ++k) {
        if (k < nk && (k < 1 || k > 4)) {
            const double t = vs::wave_sum_d(s[k]);
            if (lane == 0) red[wv][k] = t;
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < nk) {
        const int k = threadIdx.x, j = k >= 1 && k <= 4 ? k + 14 : k;
        const double t = (red[0][j] + red[1][j]) + (red[2][j] + red[3][j]);
        out[k] = j != k ? 2.0 * t : t;
    }
}

// One workgroup per pair: the sum of its tiles' partials, in a fixed order, to the state's nxt
// (refinement; stopped pairs are skipped) or to out[item * astride + k] (k >= nk written as 0).
__global__ __launch_bounds__(256) void photo_reduce_kernel(const double* __restrict__ part, int tiles, int nk,
                                                           PhotoState* state, double* out, int64_t astride)
{
    __shared__ double red[4][NACC];
    const int item = blockIdx.x;
    if (state && state[item].stopped) return;
    double* dst = state ? state[item].nxt : out + item * astride;
    const double* src = part + (int64_t)item * tiles * NACC;
    double s[NACC];
#pragma unroll
    for (int k = 0; k < NACC; ++k) s[k] = 0.0;
    for (int t = threadIdx.x; t < tiles; t += 256) {
#pragma unroll
        for (int k = 0; k < NACC; ++k)
            if (k < nk) s[k] += src[(int64_t)t * NACC + k];
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NACC; ++k) {
        if (k < nk) {
            const double t = vs::wave_sum_d(s[k]);
            if (lane == 0) red[wv][k] = t;
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < NACC) {
        const int k = threadIdx.x;
        dst[k] = k < nk ? (red[0][k] + red[1][k]) + (red[2][k] + red[3][k]) : 0.0;
    }
}

__global__ void zero_kernel(double* p, int64_t stride, int per, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * per) return;
    const int item = i / per, k = i - item * per;
    p[item * stride + k] = 0.0;
}

// Cholesky solve of the SPD 4x4 system in upper-triangle storage for -rhs; false if not positive.
__device__ bool chol_solve_neg(const double* up, const double* rhs, double* x)
{
    double A[4][4];
    int t = 0;
    for (int i = 0; i < 4; ++i)
        for (int j = i; j < 4; ++j) {
            A[i][j] = up[t];
            A[j][i] = up[t];
            ++t;
        }
    double L[4][4] = {};
    for (int j = 0; j < 4; ++j) {
        double d = A[j][j];
        for (int k = 0; k < j; ++k) d -= L[j][k] * L[j][k];
        if (!(d > 0.0)) return false;
        L[j][j] = sqrt(d);
        for (int i = j + 1; i < 4; ++i) {
            double s = A[i][j];
            for (int k = 0; k < j; ++k) s -= L[i][k] * L[j][k];
            L[i][j] = s / L[j][j];
        }
    }
    double z[4];
    for (int i = 0; i < 4; ++i) {
        double s = -rhs[i];
        for (int k = 0; k < i; ++k) s -= L[i][k] * z[k];
        z[i] = s / L[i][i];
    }
    for (int i = 3; i >= 0; --i) {
        double s = z[i];
        for (int k = i + 1; k < 4; ++k) s -= L[k][i] * x[k];
        x[i] = s / L[i][i];
    }
    return true;
}

__device__ void propose(PhotoState& s)
{
    double delta[4];
    if (!chol_solve_neg(s.cur + 5, s.cur + 15, delta)) {
        s.stopped = 1;
        return;
    }
    for (int k = 0; k < 4; ++k) s.cand[k] = s.theta[k] + delta[k];
    for (int k = 0; k < NACC; ++k) s.nxt[k] = 0.0;
}

// start: theta = theta0, candidate = theta0 (its pass gives the sums at theta0). With fit_kind the
// inputs are fitted similarities (A, B, TX, TY) in centred coordinates: theta = (rho (A-1), rho B, TX, TY).
// Pairs whose skip flag is set are stopped before any pass and keep their parameters.
__global__ void refine_init_kernel(PhotoState* st, const double* theta0, int64_t tstride, int n, int fit_kind, double rho,
                                   const int32_t* skip, int64_t skip_stride)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    PhotoState& s = st[i];
    const double* p = theta0 + i * tstride;
    double th[4] = {p[0], p[1], p[2], p[3]};
    if (fit_kind) {
        th[0] = rho * (p[0] - 1.0);
        th[1] = rho * p[1];
    }
    for (int k = 0; k < 4; ++k) s.theta[k] = s.cand[k] = th[k];
    for (int k = 0; k < NACC; ++k) s.cur[k] = s.nxt[k] = 0.0;
    s.loss0 = 0.0;
    s.stopped = (skip != nullptr && skip[i * skip_stride] != 0) ? 1 : 0;
    s.accepted = 0;
}

// after the pass at theta0: take its sums, propose the first candidate
__global__ void refine_first_kernel(PhotoState* st, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    PhotoState& s = st[i];
    if (s.stopped) return;
    for (int k = 0; k < NACC; ++k) s.cur[k] = s.nxt[k];
    s.loss0 = s.cur[0];
    propose(s);
}

// after a pass at the candidate: accept if the loss decreased, then propose the next candidate
__global__ void refine_step_kernel(PhotoState* st, int n, int last)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    PhotoState& s = st[i];
    if (s.stopped) return;
    if (!(s.nxt[0] < s.cur[0])) {
        s.stopped = 1;
        return;
    }
    for (int k = 0; k < 4; ++k) s.theta[k] = s.cand[k];
    for (int k = 0; k < NACC; ++k) s.cur[k] = s.nxt[k];
    ++s.accepted;
    if (last) {
        s.stopped = 1;
        return;
    }
    propose(s);
}

__global__ void refine_out_kernel(const PhotoState* st, int n, double* theta_out, int64_t tstride, double* loss_out,
                                  int32_t* accepted, int fit_kind, double rho)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const PhotoState& s = st[i];
    double* o = theta_out + i * tstride;
    for (int k = 0; k < 4; ++k) o[k] = s.theta[k];
    if (fit_kind) {
        o[0] = 1.0 + s.theta[0] / rho;
        o[1] = s.theta[1] / rho;
    }
    if (loss_out) {
        loss_out[2 * i] = s.loss0;
        loss_out[2 * i + 1] = s.cur[0];
    }
    if (accepted) accepted[i] = s.accepted;
}

// one wave per point; point i of the call belongs to pair i / m
__global__ __launch_bounds__(64) void photo_feature_kernel(const uint8_t* __restrict__ prev, const uint8_t* __restrict__ next,
                                                           int64_t fstride, int W, int H, int pitch, int m,
                                                           const float* __restrict__ u, const float* __restrict__ d, int hw,
                                                           double* loss, double* grad)
{
    const int64_t i = blockIdx.x;
    const int lane = threadIdx.x;
    const int64_t pair = i / m;
    const Frame F0{prev + pair * fstride, W, H, pitch}, F1{next + pair * fstride, W, H, pitch};
    const double ux = u[2 * i], uy = u[2 * i + 1];
    const double vx = ux + (double)d[2 * i], vy = uy + (double)d[2 * i + 1];
    const int side = 2 * hw + 1, nwin = side * side;
    double l = 0.0, g0 = 0.0, g1 = 0.0;
    for (int k = lane; k < nwin; k += 64) {
        const int qy = k / side - hw, qx = k % side - hw;
        double s1, gx, gy;
        sample_grad(F1, vx + qx, vy + qy, s1, gx, gy);
        const double r = s1 - sample(F0, ux + qx, uy + qy);
        l = fma(r, r, l);
        g0 = fma(2.0 * r, gx, g0);
        g1 = fma(2.0 * r, gy, g1);
    }
    l = vs::wave_sum_d(l);
    g0 = vs::wave_sum_d(g0);
    g1 = vs::wave_sum_d(g1);
    if (lane == 0) {
        loss[i] = l;
        if (grad) {
            grad[2 * i] = g0;
            grad[2 * i + 1] = g1;
        }
    }
}

int check_common(const uint8_t* prev, const uint8_t* next, int32_t w, int32_t h, int32_t pitch, int32_t n,
                 int64_t fstride, const vs_rect* om, const char* who)
{
    if (n < 0 || w <= 0 || h <= 0 || pitch < w) return vs::set_error(VS_ERR_INVALID, "%s: bad size", who);
    if (!om) return vs::set_error(VS_ERR_INVALID, "%s: null omega", who);
    if (n > 0 && (!prev || !next)) return vs::set_error(VS_ERR_INVALID, "%s: null frame", who);
    if (n > 65535) return vs::set_error(VS_ERR_INVALID, "%s: more than 65535 items", who);
    if (n > 1 && fstride < (int64_t)pitch * h) return vs::set_error(VS_ERR_INVALID, "%s: frame stride overlaps items", who);
    if (om->x0 < 0 || om->y0 < 0 || om->x1 > w || om->y1 > h)
        return vs::set_error(VS_ERR_INVALID, "%s: omega outside the frame", who);
    return VS_OK;
}

void sums_grid(const vs_rect* om, int& tiles_x, int& tiles_y)
{
    const int ow = om->x1 > om->x0 ? om->x1 - om->x0 : 0, oh = om->y1 > om->y0 ? om->y1 - om->y0 : 0;
    tiles_x = (ow + TW - 1) / TW;
    tiles_y = (oh + TH - 1) / TH;
}

// Workspace: the tiles' partial sums of every pair (room for tiles covering the whole frame), then
// the refinement states.
size_t part_bytes(int32_t n, int32_t w, int32_t h)
{
    const size_t tiles = (size_t)((w + TW - 1) / TW) * (size_t)((h + TH - 1) / TH);
    return ((size_t)n * tiles * NACC * sizeof(double) + 255) & ~(size_t)255;
}

int check_workspace(const void* ws, size_t ws_bytes, int32_t n, int32_t w, int32_t h, const char* who)
{
    const size_t need = vs_photometric_workspace(n, w, h);
    if (!ws) return vs::set_error(VS_ERR_INVALID, "%s: null workspace", who);
    if (ws_bytes < need) return vs::set_error(VS_ERR_WORKSPACE, "%s: workspace %zu < %zu", who, ws_bytes, need);
    if (reinterpret_cast<uintptr_t>(ws) & 255) return vs::set_error(VS_ERR_INVALID, "%s: workspace must be 256-byte aligned", who);
    return VS_OK;
}

}  // namespace

namespace {

int photometric_sums(const uint8_t* prev, const uint8_t* next, int64_t frame_stride, int32_t width, int32_t height,
                     int32_t pitch, int32_t n, const double* theta, int64_t theta_stride, double cx, double cy, double rho,
                     const vs_rect* omega, int need_grad, double* out, void* workspace, size_t ws_bytes, void* stream)
{
    const char* who = need_grad ? "vs_photometric_bwd" : "vs_photometric_fwd";
    int e = check_common(prev, next, width, height, pitch, n, frame_stride, omega, who);
    if (e) return e;
    if (n == 0) return VS_OK;
    if (!theta || !out) return vs::set_error(VS_ERR_INVALID, "%s: null argument", who);
    if (n > 1 && theta_stride < 4) return vs::set_error(VS_ERR_INVALID, "%s: theta stride < 4", who);
    if (!(rho > 0.0)) return vs::set_error(VS_ERR_INVALID, "%s: rho must be positive", who);
    if ((e = check_workspace(workspace, ws_bytes, n, width, height, who))) return e;
    hipStream_t s = vs::as_stream(stream);
    int tiles_x, tiles_y;
    sums_grid(omega, tiles_x, tiles_y);
    if (tiles_x * tiles_y == 0) {
        zero_kernel<<<(n * VS_PHOTO_SUMS + 255) / 256, 256, 0, s>>>(out, VS_PHOTO_SUMS, VS_PHOTO_SUMS, n);
        return vs::check_launch(who);
    }
    double* part = static_cast<double*>(workspace);
    photo_sums_kernel<<<(unsigned)(n * tiles_x * tiles_y), 256, 0, s>>>(
        prev, next, frame_stride, width, height, pitch, theta, theta_stride, nullptr, cx, cy, rho, omega->x0, omega->y0,
        omega->x1, omega->y1, need_grad != 0, part, tiles_x, tiles_y);
    if ((e = vs::check_launch(who))) return e;
    photo_reduce_kernel<<<n, 256, 0, s>>>(part, tiles_x * tiles_y, need_grad ? NACC : 1, nullptr, out, VS_PHOTO_SUMS);
    return vs::check_launch(who);
}

}  // namespace

extern "C" int vs_photometric_fwd(const uint8_t* prev, const uint8_t* next, int64_t frame_stride, int32_t width,
                                  int32_t height, int32_t pitch, int32_t n, const double* theta, int64_t theta_stride,
                                  double cx, double cy, double rho, const vs_rect* omega, double* sums, void* workspace,
                                  size_t ws_bytes, void* stream)
{
    return photometric_sums(prev, next, frame_stride, width, height, pitch, n, theta, theta_stride, cx, cy, rho, omega, 0,
                            sums, workspace, ws_bytes, stream);
}

extern "C" int vs_photometric_bwd(const uint8_t* prev, const uint8_t* next, int64_t frame_stride, int32_t width,
                                  int32_t height, int32_t pitch, int32_t n, const double* theta, int64_t theta_stride,
                                  double cx, double cy, double rho, const vs_rect* omega, double* sums, void* workspace,
                                  size_t ws_bytes, void* stream)
{
    return photometric_sums(prev, next, frame_stride, width, height, pitch, n, theta, theta_stride, cx, cy, rho, omega, 1,
                            sums, workspace, ws_bytes, stream);
}

extern "C" int vs_photometric_features(const uint8_t* prev, const uint8_t* next, int64_t frame_stride, int32_t width,
                                       int32_t height, int32_t pitch, int32_t n, const float* u, const float* d, int32_t m,
                                       int32_t win_half, double* loss, double* grad, void* stream)
{
    const char* who = "vs_photometric_features";
    if (m < 0 || n < 0 || width <= 0 || height <= 0 || pitch < width) return vs::set_error(VS_ERR_INVALID, "%s: bad size", who);
    if (win_half < 0 || win_half > 31) return vs::set_error(VS_ERR_INVALID, "%s: win_half 0..31", who);
    if (m == 0 || n == 0) return VS_OK;
    if (!prev || !next || !u || !d || !loss) return vs::set_error(VS_ERR_INVALID, "%s: null argument", who);
    if (n > 1 && frame_stride < (int64_t)pitch * height) return vs::set_error(VS_ERR_INVALID, "%s: frame stride overlaps items", who);
    if ((int64_t)n * m > 0x7fffffff) return vs::set_error(VS_ERR_INVALID, "%s: too many points", who);
    photo_feature_kernel<<<(unsigned)((int64_t)n * m), 64, 0, vs::as_stream(stream)>>>(prev, next, frame_stride, width, height,
                                                                                       pitch, m, u, d, win_half, loss, grad);
    return vs::check_launch(who);
}

extern "C" size_t vs_photometric_workspace(int32_t n, int32_t width, int32_t height)
{
    if (n <= 0 || width <= 0 || height <= 0) return 0;
    return part_bytes(n, width, height) + sizeof(PhotoState) * (size_t)n;
}

extern "C" int vs_photometric_refine(const uint8_t* prev, const uint8_t* next, int64_t frame_stride, int32_t width,
                                     int32_t height, int32_t pitch, int32_t n, const double* theta0, double* theta_out,
                                     int64_t theta_stride, int32_t param_kind, const int32_t* skip, int64_t skip_stride,
                                     double cx, double cy, double rho, const vs_rect* omega, int32_t max_steps,
                                     double* loss_out, int32_t* accepted, void* workspace, size_t ws_bytes, void* stream)
{
    int e = check_common(prev, next, width, height, pitch, n, frame_stride, omega, "vs_photometric_refine");
    if (e) return e;
    if (n == 0) return VS_OK;
    if (!theta0 || !theta_out || !workspace) return vs::set_error(VS_ERR_INVALID, "vs_photometric_refine: null argument");
    if (n > 1 && theta_stride < 4) return vs::set_error(VS_ERR_INVALID, "vs_photometric_refine: theta stride < 4");
    if (max_steps < 0 || max_steps > 100) return vs::set_error(VS_ERR_INVALID, "vs_photometric_refine: max_steps 0..100");
    if (param_kind != VS_PHOTO_THETA && param_kind != VS_PHOTO_FIT)
        return vs::set_error(VS_ERR_INVALID, "vs_photometric_refine: unknown param_kind");
    if (!(rho > 0.0)) return vs::set_error(VS_ERR_INVALID, "vs_photometric_refine: rho must be positive");
    if ((e = check_workspace(workspace, ws_bytes, n, width, height, "vs_photometric_refine"))) return e;
    hipStream_t s = vs::as_stream(stream);
    double* part = static_cast<double*>(workspace);
    PhotoState* st = reinterpret_cast<PhotoState*>(static_cast<uint8_t*>(workspace) + part_bytes(n, width, height));
    const int nb = (n + 63) / 64;
    int tiles_x, tiles_y;
    sums_grid(omega, tiles_x, tiles_y);
    const int fit_kind = param_kind == VS_PHOTO_FIT;
    refine_init_kernel<<<nb, 64, 0, s>>>(st, theta0, theta_stride, n, fit_kind, rho, skip, skip_stride);
    if ((e = vs::check_launch("vs_photometric_refine(init)"))) return e;
    auto pass = [&]() -> int {
        if (tiles_x * tiles_y == 0) return VS_OK;
        photo_sums_kernel<<<(unsigned)(n * tiles_x * tiles_y), 256, 0, s>>>(
            prev, next, frame_stride, width, height, pitch, nullptr, 0, st, cx, cy, rho, omega->x0, omega->y0, omega->x1,
            omega->y1, 1, part, tiles_x, tiles_y);
        const int e1 = vs::check_launch("vs_photometric_refine(sums)");
        if (e1) return e1;
        photo_reduce_kernel<<<n, 256, 0, s>>>(part, tiles_x * tiles_y, NACC, st, nullptr, 0);
        return vs::check_launch("vs_photometric_refine(reduce)");
    };
    if ((e = pass())) return e;
    refine_first_kernel<<<nb, 64, 0, s>>>(st, n);
    if ((e = vs::check_launch("vs_photometric_refine(first)"))) return e;
    for (int step = 0; step < max_steps; ++step) {
        if ((e = pass())) return e;
        refine_step_kernel<<<nb, 64, 0, s>>>(st, n, step == max_steps - 1);
        if ((e = vs::check_launch("vs_photometric_refine(step)"))) return e;
    }
    refine_out_kernel<<<nb, 64, 0, s>>>(st, n, theta_out, theta_stride, loss_out, accepted, fit_kind, rho);
    return vs::check_launch("vs_photometric_refine(out)");
}
