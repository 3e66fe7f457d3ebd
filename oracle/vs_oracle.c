/*
 * vs_oracle.c -- plain, slow, single-threaded CPU oracle of the stabilization hot path of
 * Lim et al., "Real-Time Optical flow-based Video Stabilization for Unmanned Aerial Vehicles"
 * (arXiv 1701.03572).
 *
 * TEST INFRASTRUCTURE ONLY. Only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library. It shares no code, header, table or constant generator with
 * the HIP library; neither includes the other.
 *
 * Arithmetic is IEEE binary64 (integers where stated), built with -ffp-contract=off so that every
 * floating-point operation below is one correctly rounded IEEE operation in the order written.
 *
 * Where the paper is silent, the reading taken is stated at each function; every reading is also
 * listed in the design notes of the repository.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define VSO_EXPORT __attribute__((visibility("default")))

static int imin(int a, int b) { return a < b ? a : b; }
static int imax(int a, int b) { return a > b ? a : b; }
static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* =============================================================================================
 * O-1  Gaussian pyramid (Section 3.2: pyramids of Adelson et al. and Bouguet make large motion
 *      small). Reading: the binomial 5-tap kernel [1 4 6 4 1]/16 in both directions, applied as
 *      ONE direct 5x5 integer sum with a single round-half-up at the end, reflect-101 borders,
 *      decimation keeping the even samples, ceil-halved sizes.
 * ============================================================================================= */
static int refl101(int t, int n)
{
    if (t < 0) t = -t;
    if (t >= n) t = 2 * n - 2 - t;
    return t;
}

VSO_EXPORT void vso_pyr_down(const uint8_t* src, int w, int h, int src_pitch, uint8_t* dst, int dst_pitch)
{
    static const int k[5] = {1, 4, 6, 4, 1};
    const int w2 = (w + 1) / 2, h2 = (h + 1) / 2;
    for (int y = 0; y < h2; ++y) {
        for (int x = 0; x < w2; ++x) {
            uint32_t acc = 0;
            for (int j = -2; j <= 2; ++j) {
                const int sy = refl101(2 * y + j, h);
                for (int i = -2; i <= 2; ++i) {
                    const int sx = refl101(2 * x + i, w);
                    acc += (uint32_t)(k[i + 2] * k[j + 2]) * src[(size_t)sy * src_pitch + sx];
                }
            }
            dst[(size_t)y * dst_pitch + x] = (uint8_t)((acc + 128u) >> 8);
        }
    }
}

/* =============================================================================================
 * O-2  Shi-Tomasi corner detection (Section 3.1, Eq. 2: R = min(lambda1, lambda2) of the
 *      windowed structure tensor; corner budget; reduced region of interest).
 *      Readings: Sobel gradients; a 3x3 rectangular window; lambda_min evaluated as
 *      2 det / (tr + sqrt(disc)) from exact 64-bit integer det/tr/disc; 3x3 non-maximum
 *      suppression inside the ROI; quality threshold q * lambda_max; total order
 *      (lambda desc, y asc, x asc); greedy minimum-distance acceptance; stop at K.
 * ============================================================================================= */
static void tensor_at(const uint8_t* im, int pitch, int x, int y, int64_t* A, int64_t* B, int64_t* C)
{
    int64_t a = 0, b = 0, c = 0;
    for (int by = -1; by <= 1; ++by) {
        for (int bx = -1; bx <= 1; ++bx) {
            const int px = x + bx, py = y + by;
            int gx = 0, gy = 0;
            /* Sobel: horizontal difference smoothed (1,2,1) vertically, and the transpose */
            for (int j = -1; j <= 1; ++j) {
                const int wj = (j == 0) ? 2 : 1;
                gx += wj * ((int)im[(size_t)(py + j) * pitch + px + 1] - (int)im[(size_t)(py + j) * pitch + px - 1]);
                gy += wj * ((int)im[(size_t)(py + 1) * pitch + px + j] - (int)im[(size_t)(py - 1) * pitch + px + j]);
            }
            a += (int64_t)gx * gx;
            b += (int64_t)gx * gy;
            c += (int64_t)gy * gy;
        }
    }
    *A = a; *B = b; *C = c;
}

static double min_eig_from_tensor(int64_t A, int64_t B, int64_t C)
{
    const int64_t det = A * C - B * B;
    const int64_t tr = A + C;
    const int64_t disc = (A - C) * (A - C) + 4 * B * B;
    if (tr == 0) return 0.0;
    /* (tr - sqrt(disc)) / 2 written without cancellation */
    return (2.0 * (double)det) / ((double)tr + sqrt((double)disc));
}

/* lambda_min of the 3x3-windowed Sobel tensor at every pixel of [x0,x1) x [y0,y1); the rectangle
 * must keep 2 pixels from every image edge. */
VSO_EXPORT void vso_min_eig_map(const uint8_t* im, int w, int h, int pitch, int x0, int y0, int x1, int y1,
                                double* out)
{
    (void)w; (void)h;
    const int ow = x1 - x0;
    for (int y = y0; y < y1; ++y)
        for (int x = x0; x < x1; ++x) {
            int64_t A, B, C;
            tensor_at(im, pitch, x, y, &A, &B, &C);
            out[(size_t)(y - y0) * ow + (x - x0)] = min_eig_from_tensor(A, B, C);
        }
}

/* integer tensor map, for pins that check the eigenvalue against a library eigensolver */
VSO_EXPORT void vso_tensor_map(const uint8_t* im, int w, int h, int pitch, int x0, int y0, int x1, int y1,
                               int64_t* out3)
{
    (void)w; (void)h;
    const int ow = x1 - x0;
    for (int y = y0; y < y1; ++y)
        for (int x = x0; x < x1; ++x) {
            int64_t* o = out3 + 3 * ((size_t)(y - y0) * ow + (x - x0));
            tensor_at(im, pitch, x, y, &o[0], &o[1], &o[2]);
        }
}

typedef struct {
    double lam;
    int x, y;
} cand_t;

static int cand_cmp(const void* pa, const void* pb)
{
    const cand_t* a = (const cand_t*)pa;
    const cand_t* b = (const cand_t*)pb;
    if (a->lam > b->lam) return -1;
    if (a->lam < b->lam) return 1;
    if (a->y != b->y) return a->y < b->y ? -1 : 1;
    if (a->x != b->x) return a->x < b->x ? -1 : 1;
    return 0;
}

/* Greedy minimum-distance acceptance over candidates already in the total order. */
VSO_EXPORT int vso_greedy_select(const int* xs, const int* ys, int n, int K, int min_dist, int* accepted_idx)
{
    const int64_t d2 = (int64_t)min_dist * min_dist;
    int na = 0;
    for (int i = 0; i < n && na < K; ++i) {
        int ok = 1;
        for (int a = 0; a < na; ++a) {
            const int64_t dx = xs[i] - xs[accepted_idx[a]];
            const int64_t dy = ys[i] - ys[accepted_idx[a]];
            if (dx * dx + dy * dy < d2) { ok = 0; break; }
        }
        if (ok) accepted_idx[na++] = i;
    }
    return na;
}

/* Returns the number of accepted corners (<= K). xy_out[2k], score_out[k]. n_cand_out (may be
 * NULL) receives the number of candidates that passed NMS and the quality threshold. */
VSO_EXPORT int vso_detect(const uint8_t* im, int w, int h, int pitch, int K, double quality, int min_dist,
                          int roi_mx, int roi_my, double* xy_out, double* score_out, int* n_cand_out)
{
    const int x0 = roi_mx, y0 = roi_my, x1 = w - roi_mx, y1 = h - roi_my;
    if (n_cand_out) *n_cand_out = 0;
    if (x1 <= x0 || y1 <= y0 || K <= 0) return 0;
    const int rw = x1 - x0, rh = y1 - y0;
    double* lam = (double*)malloc(sizeof(double) * (size_t)rw * rh);
    vso_min_eig_map(im, w, h, pitch, x0, y0, x1, y1, lam);
    double lmax = 0.0;
    for (size_t i = 0; i < (size_t)rw * rh; ++i) lmax = lam[i] > lmax ? lam[i] : lmax;
    const double thr = quality * lmax;
    cand_t* cs = (cand_t*)malloc(sizeof(cand_t) * (size_t)rw * rh);
    int nc = 0;
    for (int y = 0; y < rh; ++y) {
        for (int x = 0; x < rw; ++x) {
            const double v = lam[(size_t)y * rw + x];
            if (!(v > 0.0) || v < thr) continue;
            int is_max = 1;
            for (int dy = -1; dy <= 1 && is_max; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    if (!dx && !dy) continue;
                    const int nx = x + dx, ny = y + dy;
                    if (nx < 0 || ny < 0 || nx >= rw || ny >= rh) continue; /* outside the ROI: ignored */
                    if (lam[(size_t)ny * rw + nx] > v) { is_max = 0; break; }
                }
            if (!is_max) continue;
            cs[nc].lam = v;
            cs[nc].x = x + x0;
            cs[nc].y = y + y0;
            ++nc;
        }
    }
    qsort(cs, (size_t)nc, sizeof(cand_t), cand_cmp);
    int* xs = (int*)malloc(sizeof(int) * (size_t)(nc + 1));
    int* ys = (int*)malloc(sizeof(int) * (size_t)(nc + 1));
    int* acc = (int*)malloc(sizeof(int) * (size_t)(K + 1));
    for (int i = 0; i < nc; ++i) { xs[i] = cs[i].x; ys[i] = cs[i].y; }
    const int na = vso_greedy_select(xs, ys, nc, K, min_dist, acc);
    for (int a = 0; a < na; ++a) {
        xy_out[2 * a] = (double)cs[acc[a]].x;
        xy_out[2 * a + 1] = (double)cs[acc[a]].y;
        score_out[a] = cs[acc[a]].lam;
    }
    if (n_cand_out) *n_cand_out = nc;
    free(acc); free(ys); free(xs); free(cs); free(lam);
    return na;
}

/* =============================================================================================
 * O-3  Pyramidal Lucas-Kanade tracking with forward-backward weeding (Section 3.2, Eqs. 3-6:
 *      brightness constancy linearised to fx u + fy v + ft = 0, solved over a window by
 *      Lucas-Kanade; pyramids turn large motion into small motion; tracked points become the
 *      previous points of the next step; Section 4.1: the backward flow check weeds bad matches).
 *      Readings: images extended past their border by edge replication; derivatives are
 *      half central differences of the extended image; samples are bilinear; the window is
 *      (2 hw + 1)^2; the update solves G eta = sum (I - J) grad I; iteration stops when
 *      |eta| < eps or after max_iter; a level whose window tensor has lambda_min / N below
 *      min_eig contributes no update (and marks the point lost at level 0); a point whose final
 *      position leaves [0, W-1] x [0, H-1] is lost; the backward pass starts with zero guess.
 * ============================================================================================= */
typedef struct {
    const uint8_t* p;
    int w, h, pitch;
} img_t;

static double px_ext(const img_t* im, int x, int y)
{
    return (double)im->p[(size_t)clampi(y, 0, im->h - 1) * im->pitch + clampi(x, 0, im->w - 1)];
}

/* kind 0: intensity, 1: d/dx, 2: d/dy of the extended image at integer (x, y) */
static double field(const img_t* im, int kind, int x, int y)
{
    if (kind == 0) return px_ext(im, x, y);
    if (kind == 1) return 0.5 * (px_ext(im, x + 1, y) - px_ext(im, x - 1, y));
    return 0.5 * (px_ext(im, x, y + 1) - px_ext(im, x, y - 1));
}

static double bilinear(const img_t* im, int kind, double x, double y)
{
    const double fx = floor(x), fy = floor(y);
    const int x0 = (int)fx, y0 = (int)fy;
    const double a = x - fx, b = y - fy;
    const double v00 = field(im, kind, x0, y0), v10 = field(im, kind, x0 + 1, y0);
    const double v01 = field(im, kind, x0, y0 + 1), v11 = field(im, kind, x0 + 1, y0 + 1);
    return (1.0 - b) * ((1.0 - a) * v00 + a * v10) + b * ((1.0 - a) * v01 + a * v11);
}

typedef struct {
    int win_half;
    int max_iter;
    double eps;
    double min_eig;
    int fb;
    double fb_thresh;
} vso_lk_params;

/* One coarse-to-fine track of point u from pyramid A to pyramid B. Returns 1 if valid. */
static int lk_one(const img_t* A, const img_t* B, int levels, const vso_lk_params* p, double ux, double uy,
                  double* vx, double* vy, int* iters_l0, double* eig_margin)
{
    const int hw = p->win_half;
    const double nwin = (double)((2 * hw + 1) * (2 * hw + 1));
    double gx = 0.0, gy = 0.0;
    int ok = 1;
    *iters_l0 = 0;
    for (int l = levels - 1; l >= 0; --l) {
        const double sc = ldexp(1.0, -l);
        const double cx = ux * sc, cy = uy * sc;
        double g11 = 0, g12 = 0, g22 = 0;
        for (int qy = -hw; qy <= hw; ++qy)
            for (int qx = -hw; qx <= hw; ++qx) {
                const double ix = bilinear(&A[l], 1, cx + qx, cy + qy);
                const double iy = bilinear(&A[l], 2, cx + qx, cy + qy);
                g11 += ix * ix;
                g12 += ix * iy;
                g22 += iy * iy;
            }
        const double lmin = 0.5 * ((g11 + g22) - sqrt((g11 - g22) * (g11 - g22) + 4.0 * g12 * g12));
        /* distance of this level's test statistic from its threshold, relative to the threshold
         * (reported only: lets a caller tell decisions taken on the threshold's edge) */
        const double margin = fabs(lmin / nwin - p->min_eig) / p->min_eig;
        if (margin < *eig_margin) *eig_margin = margin;
        double nux = 0.0, nuy = 0.0;
        if (lmin / nwin < p->min_eig) {
            if (l == 0) ok = 0;
        } else {
            const double det = g11 * g22 - g12 * g12;
            for (int k = 1; k <= p->max_iter; ++k) {
                double b1 = 0.0, b2 = 0.0;
                for (int qy = -hw; qy <= hw; ++qy)
                    for (int qx = -hw; qx <= hw; ++qx) {
                        const double I = bilinear(&A[l], 0, cx + qx, cy + qy);
                        const double J = bilinear(&B[l], 0, cx + gx + nux + qx, cy + gy + nuy + qy);
                        const double d = I - J;
                        b1 += d * bilinear(&A[l], 1, cx + qx, cy + qy);
                        b2 += d * bilinear(&A[l], 2, cx + qx, cy + qy);
                    }
                const double ex = (g22 * b1 - g12 * b2) / det;
                const double ey = (g11 * b2 - g12 * b1) / det;
                nux += ex;
                nuy += ey;
                if (l == 0) *iters_l0 = k;
                if (ex * ex + ey * ey < p->eps * p->eps) break;
            }
        }
        if (l > 0) {
            gx = 2.0 * (gx + nux);
            gy = 2.0 * (gy + nuy);
        } else {
            *vx = ux + gx + nux;
            *vy = uy + gy + nuy;
        }
    }
    if (!(*vx >= 0.0 && *vy >= 0.0 && *vx <= (double)(A[0].w - 1) && *vy <= (double)(A[0].h - 1))) ok = 0;
    return ok;
}

/* prev_lv / next_lv: level base pointers; lw/lh/lpitch per level. alive may be NULL (all alive).
 * Outputs (n each): out_xy[2n], status[n], fb_err[n] (NaN where not computed), iters[2n]
 * (level-0 iterations of the forward and backward passes), eig_margin[n] (may be NULL: the smallest
 * |lambda_min / window size - min_eig| / min_eig over every level of both passes; +inf if none ran). */
VSO_EXPORT void vso_track_lk(const uint8_t* const* prev_lv, const uint8_t* const* next_lv, const int* lw,
                             const int* lh, const int* lpitch, int levels, const double* pts, int n,
                             const uint8_t* alive, const vso_lk_params* p, double* out_xy, uint8_t* status,
                             double* fb_err, int* iters, double* eig_margin)
{
    img_t A[16], B[16];
    for (int l = 0; l < levels; ++l) {
        A[l].p = prev_lv[l]; A[l].w = lw[l]; A[l].h = lh[l]; A[l].pitch = lpitch[l];
        B[l].p = next_lv[l]; B[l].w = lw[l]; B[l].h = lh[l]; B[l].pitch = lpitch[l];
    }
    for (int i = 0; i < n; ++i) {
        const double ux = pts[2 * i], uy = pts[2 * i + 1];
        out_xy[2 * i] = ux;
        out_xy[2 * i + 1] = uy;
        status[i] = 0;
        fb_err[i] = NAN;
        iters[2 * i] = iters[2 * i + 1] = 0;
        double margin = INFINITY;
        if (eig_margin) eig_margin[i] = INFINITY;
        if (alive && !alive[i]) continue;
        double vx = ux, vy = uy;
        int it0 = 0, it1 = 0;
        int ok = lk_one(A, B, levels, p, ux, uy, &vx, &vy, &it0, &margin);
        out_xy[2 * i] = vx;
        out_xy[2 * i + 1] = vy;
        iters[2 * i] = it0;
        if (ok && p->fb) {
            double bx = vx, by = vy;
            const int okb = lk_one(B, A, levels, p, vx, vy, &bx, &by, &it1, &margin);
            iters[2 * i + 1] = it1;
            const double e = sqrt((bx - ux) * (bx - ux) + (by - uy) * (by - uy));
            fb_err[i] = e;
            ok = okb && (e <= p->fb_thresh);
        }
        status[i] = (uint8_t)ok;
        if (eig_margin) eig_margin[i] = margin;
    }
}

/* =============================================================================================
 * O-4  Robust rigid / similarity fit with the hybrid switch and the skip rule (Section 4,
 *      Eq. 7: least-squares transform between src and dst point sets; similarity = 4 DOF,
 *      rigid = 3 DOF with unit scale; Section 4.1: the hybrid compares the RMS residual E_r and
 *      E_s and keeps the chosen model for a dwell of 20 frames; too few points skips the frame).
 *      Readings: centred coordinates; a seeded 2-point RANSAC (SplitMix64 counter draws) scored
 *      by residual <= 1 px, best = most inliers (ties: first hypothesis), then one least-squares
 *      refit on the best inlier set; each hybrid block of `dwell` pairs decides at its first
 *      non-skipped pair by fitting both models and comparing the RMS over all valid pairs,
 *      rigid iff E_r < E_s; a pair with fewer than min_valid points is the identity + skipped.
 * ============================================================================================= */
enum { VSO_RIGID = 0, VSO_SIMILARITY = 1, VSO_HYBRID = 2, VSO_AFFINE = 3, VSO_HYBRID3 = 4 };

typedef struct {
    int32_t model;          /* VSO_RIGID, VSO_SIMILARITY or VSO_HYBRID */
    int32_t ransac_iters;   /* 0: plain least squares on all valid points */
    double inlier_thresh;   /* px */
    uint64_t seed;
    int64_t stream_id;
    int32_t min_valid;
    int32_t dwell;
    double cx, cy;          /* centring offsets, (W-1)/2 and (H-1)/2 */
} vso_fit_params;

typedef struct {
    int64_t block;
    int32_t model;
    int32_t decided;
} vso_hybrid_state;

typedef struct {
    int32_t model;          /* model of the returned parameters */
    int32_t n_valid;
    int32_t n_inliers;
    int32_t skipped;
    int32_t decided_here;   /* 1 if this pair made the block's hybrid decision */
    int32_t pad;
    double err_rigid, err_sim;   /* RMS residuals at a decision pair, else NaN */
    double err_affine;           /* RMS residual of the affine at a three-way decision pair, else NaN */
} vso_fit_info;

/* SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): output number `ctr + 1` of the generator whose
 * state starts at `seed`, i.e. the finaliser applied to seed + (ctr + 1) * golden-gamma. */
static uint64_t splitmix64_at(uint64_t seed, uint64_t ctr)
{
    uint64_t z = seed + (ctr + 1u) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

VSO_EXPORT uint64_t vso_draw(uint64_t seed, int64_t stream_id, int64_t pair_index, int h, int k)
{
    const uint64_t ctr = (((uint64_t)stream_id & 0xFFFFFull) << 44) | (((uint64_t)pair_index & 0xFFFFFFFull) << 16) |
                         (((uint64_t)h & 0x7FFFull) << 1) | ((uint64_t)k & 1u);
    return splitmix64_at(seed, ctr);
}

/* residual^2 of dst against the model (ar, ai, br, bi) applied to src: the fixed operation order
 * px = (ar x - ai y) + br, py = (ai x + ar y) + bi. */
static double resid2(double ar, double ai, double br, double bi, double x, double y, double xd, double yd)
{
    const double px = (ar * x - ai * y) + br;
    const double py = (ai * x + ar * y) + bi;
    const double dx = xd - px, dy = yd - py;
    return dx * dx + dy * dy;
}

/* least squares over the points with mask[i] (all if mask == NULL): centroid closed forms. */
static void ls_fit(int model, const double* xs, const double* ys, const double* xd, const double* yd,
                   const uint8_t* mask, int n, double out[4])
{
    double sx = 0, sy = 0, sxd = 0, syd = 0;
    int m = 0;
    for (int i = 0; i < n; ++i) {
        if (mask && !mask[i]) continue;
        sx += xs[i]; sy += ys[i]; sxd += xd[i]; syd += yd[i];
        ++m;
    }
    const double mx = sx / m, my = sy / m, mxd = sxd / m, myd = syd / m;
    double sdot = 0, scross = 0, snorm = 0;
    for (int i = 0; i < n; ++i) {
        if (mask && !mask[i]) continue;
        const double x = xs[i] - mx, y = ys[i] - my, u = xd[i] - mxd, v = yd[i] - myd;
        sdot += x * u + y * v;
        scross += x * v - y * u;
        snorm += x * x + y * y;
    }
    double a, b;
    if (model == VSO_RIGID) {
        const double th = atan2(scross, sdot);
        a = cos(th);
        b = sin(th);
    } else if (snorm > 0.0) {
        a = sdot / snorm;
        b = scross / snorm;
    } else {
        a = 1.0;
        b = 0.0;
    }
    out[0] = a;
    out[1] = b;
    out[2] = mxd - (a * mx - b * my);
    out[3] = myd - (b * mx + a * my);
}

static double rms_all(const double p[4], const double* xs, const double* ys, const double* xd, const double* yd,
                      int n)
{
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += resid2(p[0], p[1], p[2], p[3], xs[i], ys[i], xd[i], yd[i]);
    return sqrt(s / n);
}

/* robust fit of one model: returns the inlier count; inl[n] receives the inlier flags */
static int robust_fit(int model, const vso_fit_params* P, int64_t pair_index, const double* xs, const double* ys,
                      const double* xd, const double* yd, int n, double out[4], uint8_t* inl)
{
    if (P->ransac_iters <= 0) {
        for (int i = 0; i < n; ++i) inl[i] = 1;
        ls_fit(model, xs, ys, xd, yd, NULL, n, out);
        return n;
    }
    const double tau2 = P->inlier_thresh * P->inlier_thresh;
    int best = -1, best_h = -1;
    double bm[4] = {1, 0, 0, 0};
    for (int h = 0; h < P->ransac_iters; ++h) {
        const int i1 = (int)(vso_draw(P->seed, P->stream_id, pair_index, h, 0) % (uint64_t)n);
        int i2 = (int)(vso_draw(P->seed, P->stream_id, pair_index, h, 1) % (uint64_t)n);
        if (i2 == i1) i2 = (i2 + 1) % n;
        const double dzx = xs[i2] - xs[i1], dzy = ys[i2] - ys[i1];
        const double den = dzx * dzx + dzy * dzy;
        if (den < 1.0) continue;                  /* sample points closer than 1 px: no hypothesis */
        const double wx = xd[i2] - xd[i1], wy = yd[i2] - yd[i1];
        double ar = (wx * dzx + wy * dzy) / den;  /* alpha = w / dz as complex numbers */
        double ai = (wy * dzx - wx * dzy) / den;
        double br, bi;
        if (model == VSO_RIGID) {
            const double mag = sqrt(ar * ar + ai * ai);
            if (!(mag > 0.0)) continue;
            ar = ar / mag;
            ai = ai / mag;
            const double sxs = xs[i1] + xs[i2], sys = ys[i1] + ys[i2];
            const double sxd = xd[i1] + xd[i2], syd = yd[i1] + yd[i2];
            br = (sxd - (ar * sxs - ai * sys)) * 0.5;
            bi = (syd - (ai * sxs + ar * sys)) * 0.5;
        } else {
            br = xd[i1] - (ar * xs[i1] - ai * ys[i1]);
            bi = yd[i1] - (ai * xs[i1] + ar * ys[i1]);
        }
        int score = 0;
        for (int i = 0; i < n; ++i) score += resid2(ar, ai, br, bi, xs[i], ys[i], xd[i], yd[i]) <= tau2;
        if (score > best) {
            best = score;
            best_h = h;
            bm[0] = ar; bm[1] = ai; bm[2] = br; bm[3] = bi;
        }
    }
    if (best_h < 0) {       /* every sample degenerate: least squares on all points */
        for (int i = 0; i < n; ++i) inl[i] = 1;
        ls_fit(model, xs, ys, xd, yd, NULL, n, out);
        return n;
    }
    int m = 0;
    for (int i = 0; i < n; ++i) {
        inl[i] = resid2(bm[0], bm[1], bm[2], bm[3], xs[i], ys[i], xd[i], yd[i]) <= tau2;
        m += inl[i];
    }
    if (m < 2) {            /* no usable consensus: least squares on all points */
        for (int i = 0; i < n; ++i) inl[i] = 1;
        ls_fit(model, xs, ys, xd, yd, NULL, n, out);
        return n;
    }
    ls_fit(model, xs, ys, xd, yd, inl, n, out);
    return m;
}

/* ---------------------------------------------------------------------------------------------
 * O-4b The 6-DOF affine model of Eq. 7-8 as a third candidate (a later variant of the method; the
 *      paper's hybrid stops at 4 DOF, Section 4.1). Readings (project choices, the paper is silent):
 *      [A|t] minimises the sum of squared residuals of Eq. 7 over the chosen points, found here
 *      by solving the 3x3 normal equations of the row form of Eq. 8 (X = [x y 1], one system per
 *      output row) by Gaussian elimination with partial pivoting; a point set whose centred 2x2
 *      second-moment matrix is singular (det <= 1e-12 trace^2: collinear or coincident points)
 *      has no unique affine and takes the similarity least-squares fit instead. RANSAC draws 3
 *      distinct points (SplitMix64 counters with bit 15 set, so they never meet the 2-point
 *      draws of at most 8191 hypotheses), solves the affine through them exactly (skipped when
 *      |det| < 1 px^2), scores residuals <= threshold; at least 3 inliers are needed, else the
 *      least-squares fit on all points. The three-way hybrid decides rigid against similarity
 *      as the two-way one (rigid iff E_r < E_s), then takes the affine iff E_a is smaller still.
 *      The smoother stabilises 4 DOF (Section 4.1, last paragraph): an affine pair is passed on
 *      as its nearest similarity in the Frobenius norm, a = (a11 + a22)/2, b = (a21 - a12)/2,
 *      with its translation unchanged.
 * --------------------------------------------------------------------------------------------- */
VSO_EXPORT uint64_t vso_draw3(uint64_t seed, int64_t stream_id, int64_t pair_index, int h, int k)
{
    const uint64_t ctr = (((uint64_t)stream_id & 0xFFFFFull) << 44) | (((uint64_t)pair_index & 0xFFFFFFFull) << 16) |
                         0x8000u | (((uint64_t)h & 0x1FFFull) << 2) | ((uint64_t)k & 3u);
    return splitmix64_at(seed, ctr);
}

/* m = (a11, a12, tx, a21, a22, ty): x' = a11 x + a12 y + tx, y' = a21 x + a22 y + ty, fixed order */
static double aff_resid2(const double m[6], double x, double y, double xd, double yd)
{
    const double px = (m[0] * x + m[1] * y) + m[2];
    const double py = (m[3] * x + m[4] * y) + m[5];
    const double dx = xd - px, dy = yd - py;
    return dx * dx + dy * dy;
}

static void sim_to_aff(const double p[4], double m[6])
{
    m[0] = p[0]; m[1] = -p[1]; m[2] = p[2];
    m[3] = p[1]; m[4] = p[0];  m[5] = p[3];
}

/* Gaussian elimination with partial pivoting on a 3x3 system with two right-hand sides */
static void solve3x2(double A[3][3], double B[3][2], double X[3][2])
{
    for (int c = 0; c < 3; ++c) {
        int piv = c;
        for (int r = c + 1; r < 3; ++r)
            if (fabs(A[r][c]) > fabs(A[piv][c])) piv = r;
        for (int k = 0; k < 3; ++k) { const double t = A[c][k]; A[c][k] = A[piv][k]; A[piv][k] = t; }
        for (int k = 0; k < 2; ++k) { const double t = B[c][k]; B[c][k] = B[piv][k]; B[piv][k] = t; }
        for (int r = c + 1; r < 3; ++r) {
            const double f = A[r][c] / A[c][c];
            for (int k = c; k < 3; ++k) A[r][k] -= f * A[c][k];
            for (int k = 0; k < 2; ++k) B[r][k] -= f * B[c][k];
        }
    }
    for (int k = 0; k < 2; ++k)
        for (int r = 2; r >= 0; --r) {
            double s = B[r][k];
            for (int j = r + 1; j < 3; ++j) s -= A[r][j] * X[j][k];
            X[r][k] = s / A[r][r];
        }
}

static void ls_affine(const double* xs, const double* ys, const double* xd, const double* yd, const uint8_t* mask,
                      int n, double m[6])
{
    /* degeneracy from the centred second moments */
    double sx = 0, sy = 0;
    int cnt = 0;
    for (int i = 0; i < n; ++i) {
        if (mask && !mask[i]) continue;
        sx += xs[i]; sy += ys[i]; ++cnt;
    }
    const double mx = sx / cnt, my = sy / cnt;
    double cxx = 0, cxy = 0, cyy = 0;
    for (int i = 0; i < n; ++i) {
        if (mask && !mask[i]) continue;
        const double x = xs[i] - mx, y = ys[i] - my;
        cxx += x * x; cxy += x * y; cyy += y * y;
    }
    const double tr = cxx + cyy;
    if (!(cxx * cyy - cxy * cxy > 1e-12 * tr * tr)) {
        double p[4];
        ls_fit(VSO_SIMILARITY, xs, ys, xd, yd, mask, n, p);
        sim_to_aff(p, m);
        return;
    }
    /* normal equations sum X^T X z = sum X^T y' per output row, X = [x y 1] */
    double A[3][3] = {{0}}, B[3][2] = {{0}}, Z[3][2];
    for (int i = 0; i < n; ++i) {
        if (mask && !mask[i]) continue;
        const double X[3] = {xs[i], ys[i], 1.0};
        for (int r = 0; r < 3; ++r) {
            for (int c = 0; c < 3; ++c) A[r][c] += X[r] * X[c];
            B[r][0] += X[r] * xd[i];
            B[r][1] += X[r] * yd[i];
        }
    }
    solve3x2(A, B, Z);
    m[0] = Z[0][0]; m[1] = Z[1][0]; m[2] = Z[2][0];
    m[3] = Z[0][1]; m[4] = Z[1][1]; m[5] = Z[2][1];
}

static double rms_aff(const double m[6], const double* xs, const double* ys, const double* xd, const double* yd, int n)
{
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += aff_resid2(m, xs[i], ys[i], xd[i], yd[i]);
    return sqrt(s / n);
}

/* robust affine fit: returns the inlier count; inl[n] receives the inlier flags */
static int robust_affine(const vso_fit_params* P, int64_t pair_index, const double* xs, const double* ys,
                         const double* xd, const double* yd, int n, double m[6], uint8_t* inl)
{
    const double tau2 = P->inlier_thresh * P->inlier_thresh;
    int best = -1;
    double bm[6] = {1, 0, 0, 0, 1, 0};
    for (int h = 0; P->ransac_iters > 0 && n >= 3 && h < P->ransac_iters; ++h) {
        const int i1 = (int)(vso_draw3(P->seed, P->stream_id, pair_index, h, 0) % (uint64_t)n);
        int i2 = (int)(vso_draw3(P->seed, P->stream_id, pair_index, h, 1) % (uint64_t)n);
        int i3 = (int)(vso_draw3(P->seed, P->stream_id, pair_index, h, 2) % (uint64_t)n);
        if (i2 == i1) i2 = (i2 + 1) % n;
        while (i3 == i1 || i3 == i2) i3 = (i3 + 1) % n;
        /* the affine through three points: A [p2 - p1, p3 - p1] = [q2 - q1, q3 - q1] */
        const double ex = xs[i2] - xs[i1], ey = ys[i2] - ys[i1];
        const double fx = xs[i3] - xs[i1], fy = ys[i3] - ys[i1];
        const double det = ex * fy - fx * ey;
        if (!(fabs(det) >= 1.0)) continue;
        const double gu = xd[i2] - xd[i1], gv = yd[i2] - yd[i1];
        const double hu = xd[i3] - xd[i1], hv = yd[i3] - yd[i1];
        double c[6];
        c[0] = (gu * fy - hu * ey) / det;
        c[1] = (hu * ex - gu * fx) / det;
        c[3] = (gv * fy - hv * ey) / det;
        c[4] = (hv * ex - gv * fx) / det;
        c[2] = xd[i1] - (c[0] * xs[i1] + c[1] * ys[i1]);
        c[5] = yd[i1] - (c[3] * xs[i1] + c[4] * ys[i1]);
        int score = 0;
        for (int i = 0; i < n; ++i) score += aff_resid2(c, xs[i], ys[i], xd[i], yd[i]) <= tau2;
        if (score > best) {
            best = score;
            memcpy(bm, c, sizeof(c));
        }
    }
    int cnt = 0;
    if (best >= 0) {
        for (int i = 0; i < n; ++i) {
            inl[i] = aff_resid2(bm, xs[i], ys[i], xd[i], yd[i]) <= tau2;
            cnt += inl[i];
        }
    }
    if (best < 0 || cnt < 3) {
        for (int i = 0; i < n; ++i) inl[i] = 1;
        ls_affine(xs, ys, xd, yd, NULL, n, m);
        return n;
    }
    ls_affine(xs, ys, xd, yd, inl, n, m);
    return cnt;
}

/* One pair. src/dst: 2*n_slots pixel coordinates; valid[n_slots] selects the tracked points (kept
 * in slot order). inlier_slots[n_slots] (may be NULL) receives the inlier flags per slot.
 * params4 = (a, b, tx, ty) mapping centred src to centred dst: x' = a x - b y + tx, y' = b x + a y + ty
 * (for an affine result its nearest similarity, O-4b); affine6 (may be NULL) = the returned model as
 * (a11, a12, tx, a21, a22, ty). */
VSO_EXPORT void vso_fit_pair(const double* src, const double* dst, const uint8_t* valid, int n_slots,
                             const vso_fit_params* P, int64_t pair_index, vso_hybrid_state* st, double* params4,
                             double* affine6, vso_fit_info* info, uint8_t* inlier_slots)
{
    double* xs = (double*)malloc(sizeof(double) * (size_t)(4 * n_slots + 4));
    double* ys = xs + n_slots + 1;
    double* xd = ys + n_slots + 1;
    double* yd = xd + n_slots + 1;
    int* slot = (int*)malloc(sizeof(int) * (size_t)(n_slots + 1));
    uint8_t* inl = (uint8_t*)malloc((size_t)n_slots + 1);
    uint8_t* inl2 = (uint8_t*)malloc((size_t)n_slots + 1);
    uint8_t* inl3 = (uint8_t*)malloc((size_t)n_slots + 1);
    double m6[6] = {1, 0, 0, 0, 1, 0};
    int n = 0;
    for (int i = 0; i < n_slots; ++i) {
        if (valid && !valid[i]) continue;
        xs[n] = src[2 * i] - P->cx;
        ys[n] = src[2 * i + 1] - P->cy;
        xd[n] = dst[2 * i] - P->cx;
        yd[n] = dst[2 * i + 1] - P->cy;
        slot[n] = i;
        ++n;
    }
    memset(info, 0, sizeof(*info));
    info->err_rigid = NAN;
    info->err_sim = NAN;
    info->err_affine = NAN;
    info->n_valid = n;
    if (inlier_slots) memset(inlier_slots, 0, (size_t)n_slots);
    const int hybrid = P->model == VSO_HYBRID || P->model == VSO_HYBRID3;
    const int64_t block = pair_index / (P->dwell > 0 ? P->dwell : 1);
    if (st->block != block) {
        st->block = block;
        st->decided = 0;
    }
    if (n < P->min_valid || n < 2) {
        params4[0] = 1.0; params4[1] = 0.0; params4[2] = 0.0; params4[3] = 0.0;
        info->skipped = 1;
        info->model = hybrid ? st->model : P->model;
        goto done;
    }
    int model;
    if (hybrid) {
        if (!st->decided) {
            double pr[4], ps[4], pa[6];
            const int mr = robust_fit(VSO_RIGID, P, pair_index, xs, ys, xd, yd, n, pr, inl);
            const int ms = robust_fit(VSO_SIMILARITY, P, pair_index, xs, ys, xd, yd, n, ps, inl2);
            const double er = rms_all(pr, xs, ys, xd, yd, n);
            const double es = rms_all(ps, xs, ys, xd, yd, n);
            info->err_rigid = er;
            info->err_sim = es;
            info->decided_here = 1;
            st->decided = 1;
            st->model = (er < es) ? VSO_RIGID : VSO_SIMILARITY;
            int ma = 0;
            if (P->model == VSO_HYBRID3) {
                ma = robust_affine(P, pair_index, xs, ys, xd, yd, n, pa, inl3);
                info->err_affine = rms_aff(pa, xs, ys, xd, yd, n);
                if (info->err_affine < (st->model == VSO_RIGID ? er : es)) st->model = VSO_AFFINE;
            }
            model = st->model;
            if (model == VSO_RIGID) {
                memcpy(params4, pr, sizeof(pr));
                sim_to_aff(pr, m6);
                info->n_inliers = mr;
            } else if (model == VSO_SIMILARITY) {
                memcpy(params4, ps, sizeof(ps));
                sim_to_aff(ps, m6);
                info->n_inliers = ms;
                memcpy(inl, inl2, (size_t)n);
            } else {
                memcpy(m6, pa, sizeof(pa));
                info->n_inliers = ma;
                memcpy(inl, inl3, (size_t)n);
            }
            info->model = model;
            goto write_inliers;
        }
        model = st->model;
    } else {
        model = P->model;
    }
    if (model == VSO_AFFINE) {
        info->n_inliers = robust_affine(P, pair_index, xs, ys, xd, yd, n, m6, inl);
    } else {
        info->n_inliers = robust_fit(model, P, pair_index, xs, ys, xd, yd, n, params4, inl);
        sim_to_aff(params4, m6);
    }
    info->model = model;
write_inliers:
    if (model == VSO_AFFINE) {
        params4[0] = (m6[0] + m6[4]) * 0.5;
        params4[1] = (m6[3] - m6[1]) * 0.5;
        params4[2] = m6[2];
        params4[3] = m6[5];
    }
    if (inlier_slots)
        for (int i = 0; i < n; ++i) inlier_slots[slot[i]] = inl[i];
done:
    if (affine6) memcpy(affine6, m6, sizeof(m6));
    free(inl3); free(inl2); free(inl); free(slot); free(xs);
}

/* =============================================================================================
 * O-5  Motion compensation by trajectory smoothing (Section 5.1: accumulate the per-pair
 *      parameters into a trajectory, smooth it with an averaging window twice the smoothing
 *      radius, and correct each frame by smoothed - accumulated; Section 6: a sliding store of
 *      recent parameters for the real-time version).
 *      Readings: per-pair parameters (tx, ty, angle = atan2(b, a), log-scale = ln|a + ib|);
 *      P_0 = 0, P_j = sum_{k<j}; modes: 0 centred moving average over [j-r, j+r] truncated at the
 *      ends (direct ascending sums), 1 causal mean over [j-2r, j], 2 per-parameter Kalman filter
 *      of a random walk with normalised measurement noise 1 and process noise `ratio`;
 *      correction D_j = Q_j - P_j applied as a similarity about the image centre, followed by a
 *      zoom 1/(1 - 2 crop) about the centre.
 * ============================================================================================= */
VSO_EXPORT void vso_smooth(const double* pair_params, int n_frames, int mode, int radius, double ratio,
                           double crop, double cx, double cy, double* traj, double* smooth, double* mats)
{
    /* traj/smooth: [n_frames][4]; mats: [n_frames][6] (src -> dst, pixel coordinates) */
    for (int c = 0; c < 4; ++c) traj[c] = 0.0;
    for (int j = 1; j < n_frames; ++j) {
        const double* q = pair_params + 4 * (j - 1);
        const double d[4] = {q[2], q[3], atan2(q[1], q[0]), log(sqrt(q[0] * q[0] + q[1] * q[1]))};
        for (int c = 0; c < 4; ++c) traj[4 * j + c] = traj[4 * (j - 1) + c] + d[c];
    }
    if (mode == 0 || mode == 1) {
        for (int j = 0; j < n_frames; ++j) {
            const int lo = (mode == 0) ? imax(0, j - radius) : imax(0, j - 2 * radius);
            const int hi = (mode == 0) ? imin(n_frames - 1, j + radius) : j;
            for (int c = 0; c < 4; ++c) {
                double s = 0.0;
                for (int i = lo; i <= hi; ++i) s += traj[4 * i + c];
                smooth[4 * j + c] = s / (double)(hi - lo + 1);
            }
        }
    } else {
        for (int c = 0; c < 4; ++c) {
            double x = traj[c], S = 0.0;
            smooth[c] = x;
            for (int j = 1; j < n_frames; ++j) {
                const double Sm = S + ratio;
                const double K = Sm / (Sm + 1.0);
                x = x + K * (traj[4 * j + c] - x);
                S = (1.0 - K) * Sm;
                smooth[4 * j + c] = x;
            }
        }
    }
    const double z = 1.0 / (1.0 - 2.0 * crop);
    for (int j = 0; j < n_frames; ++j) {
        const double dx = smooth[4 * j] - traj[4 * j];
        const double dy = smooth[4 * j + 1] - traj[4 * j + 1];
        const double da = smooth[4 * j + 2] - traj[4 * j + 2];
        const double ds = smooth[4 * j + 3] - traj[4 * j + 3];
        const double s = exp(ds);
        const double a = s * cos(da), b = s * sin(da);
        double* M = mats + 6 * j;
        M[0] = z * a;
        M[1] = -z * b;
        M[2] = z * (dx - a * cx + b * cy) + cx;
        M[3] = z * b;
        M[4] = z * a;
        M[5] = z * (dy - b * cx - a * cy) + cy;
    }
}

/* =============================================================================================
 * O-6  Image composition (Section 5: warp each frame by its corrected transform, with cropping
 *      to hide the unfilled area). Readings: inverse mapping, bilinear interpolation, samples
 *      outside the source take the border value, round half up, clamp to [0, 255].
 * ============================================================================================= */
VSO_EXPORT void vso_warp(const uint8_t* src, int w, int h, int pitch, const double* M, uint8_t* dst, int dpitch,
                         int border)
{
    const double det = M[0] * M[4] - M[1] * M[3];
    const double i00 = M[4] / det, i01 = -M[1] / det, i10 = -M[3] / det, i11 = M[0] / det;
    const double i02 = -(i00 * M[2] + i01 * M[5]);
    const double i12 = -(i10 * M[2] + i11 * M[5]);
    for (int y = 0; y < h; ++y) {
        for (int x = 0; x < w; ++x) {
            const double sx = i00 * x + i01 * y + i02;
            const double sy = i10 * x + i11 * y + i12;
            const double fx = floor(sx), fy = floor(sy);
            const double a = sx - fx, b = sy - fy;
            double v[4];
            for (int k = 0; k < 4; ++k) {
                const double xx = fx + (k & 1), yy = fy + (k >> 1);
                v[k] = (xx >= 0 && yy >= 0 && xx <= w - 1 && yy <= h - 1)
                           ? (double)src[(size_t)yy * pitch + (size_t)xx]
                           : (double)border;
            }
            const double val = (1.0 - b) * ((1.0 - a) * v[0] + a * v[1]) + b * ((1.0 - a) * v[2] + a * v[3]);
            double r = floor(val + 0.5);
            r = r < 0 ? 0 : (r > 255 ? 255 : r);
            dst[(size_t)y * dpitch + x] = (uint8_t)r;
        }
    }
}

/* =============================================================================================
 * O-7  Photometric loss and its gradient, and Gauss-Newton refinement of a fitted similarity.
 *      Not in the paper: a project extension that checks the fitted pair transform of Eq. 7
 *      against the image intensities (the brightness constancy of Eq. 3 applied to the whole
 *      frame) and refines it.
 *      Readings: S(F, p) is the bilinear interpolant of F extended by edge replication; its
 *      gradient is the derivative of the bilinear piece in cell floor(p) (the right derivative at
 *      integer crossings). The transform is T_theta(x) = x + [[a, -b], [b, a]] (x - c) / rho + t
 *      with theta = (a, b, tx, ty), c the frame centre and rho = max(W, H) / 2, so a fitted
 *      similarity (A, B, TX, TY) in centred coordinates is theta = (rho (A - 1), rho B, TX, TY).
 *      Global loss L_g = sum over x in the fixed rectangle Omega of (S(F1, T(x)) - F0(x))^2.
 *      Feature loss of point i with displacement d_i: sum over the (2h+1)^2 window offsets q of
 *      (S(F1, u_i + d_i + q) - S(F0, u_i + q))^2. Gauss-Newton: solve (J^T J) delta = -J^T r for the
 *      residual Jacobian J = grad S . dT/dtheta, accept theta + delta only if L_g decreases, stop
 *      at the first rejected step or after max_steps.
 * ============================================================================================= */
static void sample_d(const img_t* im, double x, double y, double* v, double* gx, double* gy)
{
    const double fx = floor(x), fy = floor(y);
    const double a = x - fx, b = y - fy;
    const int x0 = (int)fx, y0 = (int)fy;
    const double p00 = px_ext(im, x0, y0), p10 = px_ext(im, x0 + 1, y0);
    const double p01 = px_ext(im, x0, y0 + 1), p11 = px_ext(im, x0 + 1, y0 + 1);
    *v = (1.0 - a) * (1.0 - b) * p00 + a * (1.0 - b) * p10 + (1.0 - a) * b * p01 + a * b * p11;
    if (gx) *gx = (1.0 - b) * (p10 - p00) + b * (p11 - p01);
    if (gy) *gy = (1.0 - a) * (p01 - p00) + a * (p11 - p10);
}

/* out[19]: loss, grad[4] (dL/dtheta), the upper triangle of J^T J row by row (00 01 02 03 11 12 13
 * 22 23 33), J^T r[4]. */
VSO_EXPORT void vso_photo_global(const uint8_t* f0, const uint8_t* f1, int w, int h, int pitch, const double* theta,
                                 double cx, double cy, double rho, int ox0, int oy0, int ox1, int oy1, double* out)
{
    const img_t I1 = {f1, w, h, pitch};
    for (int k = 0; k < 19; ++k) out[k] = 0.0;
    for (int y = oy0; y < oy1; ++y) {
        for (int x = ox0; x < ox1; ++x) {
            const double dx = (x - cx) / rho, dy = (y - cy) / rho;
            const double tx = x + theta[0] * dx - theta[1] * dy + theta[2];
            const double ty = y + theta[1] * dx + theta[0] * dy + theta[3];
            double s, sx, sy;
            sample_d(&I1, tx, ty, &s, &sx, &sy);
            const double r = s - (double)f0[(size_t)y * pitch + x];
            /* dT/da = (dx, dy), dT/db = (-dy, dx), dT/dtx = (1, 0), dT/dty = (0, 1) */
            const double J[4] = {sx * dx + sy * dy, -sx * dy + sy * dx, sx, sy};
            out[0] += r * r;
            int t = 5;
            for (int i = 0; i < 4; ++i) {
                out[1 + i] += 2.0 * r * J[i];
                out[15 + i] += J[i] * r;
                for (int j = i; j < 4; ++j) out[t++] += J[i] * J[j];
            }
        }
    }
}

/* u, d: [m][2]; loss[m]; grad[m][2] (may be NULL) */
VSO_EXPORT void vso_photo_feature(const uint8_t* f0, const uint8_t* f1, int w, int h, int pitch, const double* u,
                                  const double* d, int m, int hw, double* loss, double* grad)
{
    const img_t I0 = {f0, w, h, pitch}, I1 = {f1, w, h, pitch};
    for (int i = 0; i < m; ++i) {
        double l = 0.0, g0 = 0.0, g1 = 0.0;
        for (int qy = -hw; qy <= hw; ++qy) {
            for (int qx = -hw; qx <= hw; ++qx) {
                double s1, sx, sy, s0;
                sample_d(&I1, u[2 * i] + d[2 * i] + qx, u[2 * i + 1] + d[2 * i + 1] + qy, &s1, &sx, &sy);
                sample_d(&I0, u[2 * i] + qx, u[2 * i + 1] + qy, &s0, NULL, NULL);
                const double r = s1 - s0;
                l += r * r;
                g0 += 2.0 * r * sx;
                g1 += 2.0 * r * sy;
            }
        }
        loss[i] = l;
        if (grad) {
            grad[2 * i] = g0;
            grad[2 * i + 1] = g1;
        }
    }
}

/* Solves the symmetric 4x4 system given by its upper triangle (as in vso_photo_global) for
 * -rhs, by Gaussian elimination with partial pivoting. Returns 0 if a pivot vanishes. */
static int solve4_neg(const double* upper, const double* rhs, double* x)
{
    double M[4][5];
    int t = 0;
    for (int i = 0; i < 4; ++i)
        for (int j = i; j < 4; ++j) {
            M[i][j] = upper[t];
            M[j][i] = upper[t];
            ++t;
        }
    for (int i = 0; i < 4; ++i) M[i][4] = -rhs[i];
    for (int c = 0; c < 4; ++c) {
        int p = c;
        for (int r = c + 1; r < 4; ++r)
            if (fabs(M[r][c]) > fabs(M[p][c])) p = r;
        if (M[p][c] == 0.0) return 0;
        if (p != c)
            for (int k = 0; k < 5; ++k) {
                const double tmp = M[c][k];
                M[c][k] = M[p][k];
                M[p][k] = tmp;
            }
        for (int r = c + 1; r < 4; ++r) {
            const double f = M[r][c] / M[c][c];
            for (int k = c; k < 5; ++k) M[r][k] -= f * M[c][k];
        }
    }
    for (int r = 3; r >= 0; --r) {
        double s = M[r][4];
        for (int k = r + 1; k < 4; ++k) s -= M[r][k] * x[k];
        x[r] = s / M[r][r];
    }
    return 1;
}

/* Returns the number of accepted steps; theta_out[4]; loss_out[2] = (initial, final). */
VSO_EXPORT int vso_photo_refine(const uint8_t* f0, const uint8_t* f1, int w, int h, int pitch, const double* theta0,
                                double cx, double cy, double rho, int ox0, int oy0, int ox1, int oy1, int max_steps,
                                double* theta_out, double* loss_out)
{
    double th[4] = {theta0[0], theta0[1], theta0[2], theta0[3]};
    double cur[19];
    vso_photo_global(f0, f1, w, h, pitch, th, cx, cy, rho, ox0, oy0, ox1, oy1, cur);
    loss_out[0] = cur[0];
    int accepted = 0;
    for (int step = 0; step < max_steps; ++step) {
        double delta[4];
        if (!solve4_neg(cur + 5, cur + 15, delta)) break;
        const double cand[4] = {th[0] + delta[0], th[1] + delta[1], th[2] + delta[2], th[3] + delta[3]};
        double nxt[19];
        vso_photo_global(f0, f1, w, h, pitch, cand, cx, cy, rho, ox0, oy0, ox1, oy1, nxt);
        if (!(nxt[0] < cur[0])) break;
        for (int k = 0; k < 4; ++k) th[k] = cand[k];
        for (int k = 0; k < 19; ++k) cur[k] = nxt[k];
        ++accepted;
    }
    for (int k = 0; k < 4; ++k) theta_out[k] = th[k];
    loss_out[1] = cur[0];
    return accepted;
}
