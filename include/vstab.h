/*
 * vstab.h -- C ABI of the MI355X (gfx950) video-stabilization hot path of
 * Lim et al., "Real-Time Optical flow-based Video Stabilization for Unmanned Aerial Vehicles"
 * (arXiv 1701.03572).
 *
 * The six operations follow the paper's three-stage pipeline (Section 2, framework figure):
 * motion estimation (pyramids, corners, optical-flow tracking, robust model fit; Sections 3-4),
 * motion compensation (trajectory smoothing; Section 5.1) and image composition (warp; Section 5).
 *
 * Conventions shared by every call
 *  - Pointers named *frames, *pyrs, xy*, score, alive, status, fb_err, n_valid, params, info,
 *    inliers, mats, state and workspace are DEVICE pointers owned by the caller. Structs passed
 *    as `const vs_*_params*` and `vs_pyramid*` are HOST pointers read during the call only.
 *  - `stream` is a hipStream_t (NULL: the null stream). Every call only enqueues work on it:
 *    no allocation, no free, no host synchronisation. Data-dependent outcomes (corner counts,
 *    skip flags, model choices, emitted frames) are written to device memory, never returned.
 *  - Images are 8-bit grayscale, row-major, `pitch` bytes per row (pitch >= width).
 *    Coordinates: x = column, y = row, pixel centres at integers; points are interleaved float
 *    pairs (x, y).
 *  - Batches: every call takes a count `n` of independent items and byte (or element) strides
 *    between them, so one launch can serve one frame, a run of frames or many streams.
 *  - Return codes: VS_OK (0), VS_ERR_INVALID (-1: null pointer, bad size, count or stride),
 *    VS_ERR_UNSUPPORTED (-2: levels > VS_MAX_LEVELS, window > 31x31, capacity > VS_MAX_CORNERS),
 *    VS_ERR_WORKSPACE (-3: workspace too small), VS_ERR_HIP (-4: launch failure; the message is
 *    available from vs_last_error()). On an error no work has been enqueued.
 */
#ifndef VSTAB_H
#define VSTAB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VS_MAX_LEVELS 8
#define VS_MAX_CORNERS 4096
#define VS_TRAJ_RING 256

enum { VS_OK = 0, VS_ERR_INVALID = -1, VS_ERR_UNSUPPORTED = -2, VS_ERR_WORKSPACE = -3, VS_ERR_HIP = -4 };
enum { VS_RIGID = 0, VS_SIMILARITY = 1, VS_HYBRID = 2, VS_AFFINE = 3, VS_HYBRID3 = 4 };
enum { VS_SMOOTH_CENTERED = 0, VS_SMOOTH_CAUSAL = 1, VS_SMOOTH_KALMAN = 2 };

/* ---------------------------------------------------------------------------------------------
 * Pyramid layout (Section 3.2: image pyramids turn large motion into small motion).
 * Level 0 is the caller's frame itself (never copied). Levels 1..levels-1 live in one pyramid
 * buffer of `bytes` bytes: level l has size width[l] x height[l] with width[l+1] =
 * (width[l] + 1) / 2 (same for height), row pitch pitch[l] (a multiple of 64) and starts at
 * byte offset[l] (a multiple of 256). pitch[0] is the frame pitch, offset[0] = 0 (unused).
 * ------------------------------------------------------------------------------------------- */
typedef struct {
    int32_t levels;
    int32_t width[VS_MAX_LEVELS];
    int32_t height[VS_MAX_LEVELS];
    int32_t pitch[VS_MAX_LEVELS];
    int64_t offset[VS_MAX_LEVELS];
    int64_t bytes;
} vs_pyramid;

/* Host only. Fills *out for a width x height frame of row pitch `pitch0`. Every level must keep
 * width and height >= 16, else VS_ERR_INVALID. */
int vs_pyramid_layout(int32_t width, int32_t height, int32_t pitch0, int32_t levels, vs_pyramid* out);

/* build_pyramid -- Section 3.2 (pyramids of Adelson et al. / Bouguet).
 * Level l+1 = even samples of level l correlated with the binomial kernel [1 4 6 4 1]^T [1 4 6 4 1]
 * / 256 (one integer sum, round half up), borders reflected without repeating the edge pixel.
 * Item i reads frames + i * frame_stride (pitch layout->pitch[0]) and writes levels 1.. into
 * pyrs + i * pyr_stride. Bit-exact. */
int vs_build_pyramid(const uint8_t* frames, int64_t frame_stride, uint8_t* pyrs, int64_t pyr_stride, int32_t n,
                     const vs_pyramid* layout, void* stream);

/* ---------------------------------------------------------------------------------------------
 * detect_corners -- Section 3.1, Eq. 2 (Shi-Tomasi score R = min(lambda1, lambda2) of the
 * windowed gradient tensor), the corner budget and the reduced region of interest.
 * Gradients are Sobel, the window is 3x3, the score is evaluated in binary64 as
 * 2 det / (tr + sqrt(disc)) from exact integer det, tr, disc. Candidates are the pixels of the ROI
 * [roi_mx, W - roi_mx) x [roi_my, H - roi_my) whose score is > 0, >= quality * (max score in the ROI)
 * and >= the score of each of their 8 neighbours inside the ROI. In the order (score desc, y asc,
 * x asc) a candidate is accepted iff its squared distance to every accepted corner is >= min_dist^2;
 * selection stops after max_corners acceptances.
 * Item i reads frames + i * frame_stride. Its per-item records sit at record index g = i * istride
 * (istride >= 1 lets a call address every 5th record of a pair-major array); each record has
 * `capacity` point slots:
 *   xy[g * capacity + k][2] (float, integer-valued), score[g * capacity + k] (double, may be NULL),
 *   count[g] (int32), alive[g * capacity + k] (uint8: 1 for the accepted slots, 0 for the rest).
 * Gating: when gate != NULL, item i runs only if gate[g] < gate_min; otherwise its outputs are
 * left untouched (this implements the re-detection after a skipped pair on the device).
 * max_corners <= capacity <= VS_MAX_CORNERS, roi margins >= 2.
 * workspace: at least vs_detect_workspace(width, height, n) bytes. */
typedef struct {
    int32_t max_corners;
    double quality;
    int32_t min_dist;
    int32_t roi_mx, roi_my;
    /* optional (device, may be NULL): item i accepts at most min(max_corners_per_item[i], max_corners)
     * corners; lets one call serve items of different corner budgets */
    const int32_t* max_corners_per_item;
} vs_detect_params;

size_t vs_detect_workspace(int32_t width, int32_t height, int32_t n);
int vs_detect_corners(const uint8_t* frames, int64_t frame_stride, int32_t width, int32_t height, int32_t pitch,
                      int32_t n, int32_t istride, const int32_t* gate, int32_t gate_min, const vs_detect_params* p,
                      int32_t capacity,
                      float* xy, double* score, int32_t* count, uint8_t* alive, void* workspace, size_t ws_bytes,
                      void* stream);

/* ---------------------------------------------------------------------------------------------
 * track_lk -- Section 3.2, Eqs. 3-6 (brightness constancy linearised to fx u + fy v + ft = 0,
 * solved over a window by Lucas-Kanade, coarse to fine over the pyramid; tracked points become
 * the previous points of the next step) and the backward consistency check of Section 4.1.
 * For every alive slot u: at each level l from the top, c = u / 2^l, samples of the edge-
 * replicated image are bilinear, gradients are half central differences; G = sum grad I grad I^T
 * over the (2 win_half + 1)^2 window; if lambda_min(G) / window_size < min_eig the level gives no
 * update (at level 0 the point is lost); otherwise nu += G^-1 sum (I - J) grad I until |eta| < eps
 * or max_iter; the guess passed down is 2 (g + nu). v = u + g + nu must lie in the image. With fb,
 * the same track from v back to the previous frame must return within fb_thresh of u.
 * FP32 arithmetic.
 * Item i uses the frame pair (prev_frames + i * frame_stride, next_frames + i * frame_stride),
 * their pyramids (prev_pyrs/next_pyrs + i * pyr_stride), and the record g = i * istride of every
 * per-item array: point slots xy_prev[g * capacity + k][2] with alive_prev[g * capacity + k].
 * Outputs: xy_next[g * capacity + k][2], status[g * capacity + k] (1 = tracked and consistent),
 * fb_err[g * capacity + k] (may be NULL; NaN where not computed), n_valid[g] (may be NULL: number
 * of status-1 slots), and optional chained copies xy_chain / alive_chain (may be NULL) receiving the
 * same values as xy_next / status (the next step's input, which a later re-detection may
 * overwrite without touching this step's outputs). xy_chain may alias xy_prev (same for alive).
 * work (may be NULL): uint64[2 * n]; work[2 i] and work[2 i + 1] are set by the call to the number
 * of window set-ups (point x level x direction) and of Gauss-Newton iterations it performed for
 * item i, for throughput accounting. */
typedef struct {
    int32_t win_half;
    int32_t max_iter;
    float eps;
    float min_eig;
    int32_t fb;
    float fb_thresh;
} vs_lk_params;

int vs_track_lk(const uint8_t* prev_frames, const uint8_t* prev_pyrs, const uint8_t* next_frames,
                const uint8_t* next_pyrs, int64_t frame_stride, int64_t pyr_stride, int32_t n, int32_t istride,
                const vs_pyramid* layout, const float* xy_prev, const uint8_t* alive_prev, int32_t capacity,
                const vs_lk_params* p, float* xy_next, uint8_t* status, float* fb_err, int32_t* n_valid,
                float* xy_chain, uint8_t* alive_chain, uint64_t* work, void* stream);

/* ---------------------------------------------------------------------------------------------
 * track_lk_segments -- the tracking of vs_track_lk (Section 3.2, Eqs. 3-6) with its backward check
 * (Section 4.1) over chains of consecutive pairs, the points tracked into a frame being the previous
 * points of the next pair (Section 3.2: features are tracked on from frame to frame between
 * re-detections every few frames). Item i is a chain: its frame s (s = 0 .. pairs_i) is at
 * frames + i * frame_stride + s * frame_step (pyramid at pyrs + i * pyr_stride + s * pyr_step), its
 * pair s = (frame s, frame s + 1) has the point records r = i * istride + s (slot k of a point array
 * at [r * capacity + k]); pairs_i = pairs for i < n - 1 and last_pairs for i = n - 1. The call tracks
 * pairs first .. pairs_i - 1 of every item whose gate lets it in (gate NULL: every item; else
 * gate[i * istride] < gate_min), starting from the points xy / alive of pair `first`, and writes for
 * each of those pairs what vs_track_lk writes with xy_chain / alive_chain set to the next pair's
 * records: dst, status, fb_err (may be NULL; NaN where not computed), n_valid[r] (may be NULL), and
 * the next pair's xy / alive (not after an item's last pair). It assumes that no pair in the chain is
 * skipped: where a pair s ends with n_valid < min_valid and frame s + 1 is detected again, a call
 * with first = s + 1 and the gate at the n_valid of pair s (gate = n_valid + s, gate_min = min_valid)
 * makes the pairs after it again from the new points; calling it for s + 1 = 1 .. pairs - 1 in
 * order, each after the gated re-detection of frame s + 1, gives exactly the records of one
 * vs_track_lk call per pair with the re-detection between them. One wave follows a point slot of an
 * item through its pairs: every frame is read by its windows around one point position, and with the
 * backward check the window set-ups of a frame (samples, gradients, tensor and eigenvalue test of
 * Eqs. 4-6) serve both the backward track of the pair ending there and the forward track of the pair
 * starting there. Results are those of vs_track_lk bit for bit.
 * work (may be NULL): uint64[3 * n], set by the call: per item, the window set-ups (point x level x
 * direction, as separate tracks would form them) and Gauss-Newton iterations of the tracks kept, and
 * the window set-ups formed (a shared one once). Forward tracks made for points that then fail the
 * check of the pair before are not counted.
 * Errors: VS_ERR_INVALID for a null layout, parameters, frame, pyramid (more than one level) or
 * point array, a negative count, istride < 1, pairs > istride, last_pairs > pairs or first < 0;
 * otherwise those of vs_track_lk. n = 0, capacity = 0 or first >= pairs enqueue nothing.
 * Device buffers are the caller's; launches are enqueued on `stream`; nothing is allocated and the
 * host is not synchronised. */
int vs_track_lk_segments(const uint8_t* frames, const uint8_t* pyrs, int64_t frame_stride, int64_t pyr_stride,
                         int64_t frame_step, int64_t pyr_step, int32_t n, int32_t istride, int32_t pairs,
                         int32_t last_pairs, int32_t first, const vs_pyramid* layout, int32_t capacity,
                         const vs_lk_params* p, float* xy, uint8_t* alive, float* dst, uint8_t* status,
                         float* fb_err, int32_t* n_valid, const int32_t* gate, int32_t gate_min, uint64_t* work,
                         void* stream);

/* ---------------------------------------------------------------------------------------------
 * fit_similarity -- Section 4, Eq. 7 (least-squares transform from src to dst points), the
 * similarity (4 DOF) and rigid (3 DOF, unit scale) models, the hybrid mechanism of Section 4.1
 * (compare the RMS residuals E_r and E_s, keep the choice for a dwell of `dwell` pairs) and the
 * skip rule (too few points: no stabilization for that pair).
 * Item i is pair index pair_index0 + i of one stream. Its valid points are the slots with
 * valid[i][k] = 1, in slot order, in centred coordinates (x - cx, y - cy). With n_valid < min_valid
 * the pair is the identity and skipped. Otherwise each model is fitted by a seeded 2-point RANSAC
 * (ransac_iters hypotheses drawn by SplitMix64 from (seed, stream_id, pair index, hypothesis),
 * scored by the count of residuals <= inlier_thresh, first best wins) followed by a binary64
 * least-squares refit on the best inlier set (ransac_iters = 0: least squares on all points).
 * HYBRID: the first non-skipped pair of each dwell block fits both models and picks rigid iff
 * E_r < E_s (RMS over all valid points); later pairs of the block use that model. *state (device,
 * one per stream) carries the block decision across calls; initialise it with
 * vs_fit_state_init. Pairs of one call must be consecutive and in order.
 * Outputs: params[i][4] = (a, b, tx, ty) with x' = a x - b y + tx, y' = b x + a y + ty (centred),
 * info[i], inliers[i][capacity] (may be NULL).
 * workspace: at least vs_fit_workspace(n, capacity) bytes. */
typedef struct {
    int32_t model;
    int32_t ransac_iters;
    double inlier_thresh;
    uint64_t seed;
    int64_t stream_id;
    int32_t min_valid;
    int32_t dwell;
    double cx, cy;
} vs_fit_params;

typedef struct {
    int64_t block;
    int32_t model;
    int32_t decided;
} vs_fit_state;

typedef struct {
    int32_t model;
    int32_t n_valid;
    int32_t n_inliers;
    int32_t skipped;
    int32_t decided_here;
    int32_t pad;
    double err_rigid;
    double err_sim;
    double err_affine;   /* VS_HYBRID3 decision pairs only, else NaN */
} vs_fit_info;

size_t vs_fit_workspace(int32_t n, int32_t capacity);
int vs_fit_state_init(vs_fit_state* state, void* stream);
int vs_fit_similarity(const float* src, const float* dst, const uint8_t* valid, int32_t capacity, int32_t n,
                      const vs_fit_params* p, int64_t pair_index0, vs_fit_state* state, double* params,
                      vs_fit_info* info, uint8_t* inliers, void* workspace, size_t ws_bytes, void* stream);

/* fit_motion -- fit_similarity extended by the 6-DOF affine [A|t] of Eq. 7-8 (the least-squares
 * 2x3 transform the paper starts from before restricting itself to 4 DOF in Section 4.1).
 * model VS_AFFINE fits the affine alone; VS_HYBRID3 makes the hybrid a three-way choice: at a
 * block's decision pair rigid is preferred over the similarity iff E_r < E_s, and the affine
 * replaces that choice iff its RMS residual E_a is smaller still. The affine's RANSAC draws 3
 * distinct points per hypothesis (SplitMix64 counters disjoint from the 2-point draws), solves the
 * affine through them exactly (no hypothesis when the sample's doubled triangle area is below
 * 1 px^2) and needs at least 3 inliers; its refit is binary64 least squares. A point set whose
 * centred second-moment matrix is singular (det <= 1e-12 trace^2) takes the similarity fit. With
 * the affine in the mode ransac_iters must be <= 8191.
 * params[i][4]: as for fit_similarity; for an affine pair its nearest similarity in the Frobenius
 * norm, a = (a11 + a22)/2, b = (a21 - a12)/2, same translation (the smoother stabilises 4 DOF).
 * affine6[i][6] (device, may be NULL): the pair's model as (a11, a12, tx, a21, a22, ty),
 * x' = a11 x + a12 y + tx, y' = a21 x + a22 y + ty in centred coordinates; the identity for a
 * skipped pair. Every other argument, the workspace size and the errors are those of
 * fit_similarity, which is fit_motion with affine6 = NULL. */
int vs_fit_motion(const float* src, const float* dst, const uint8_t* valid, int32_t capacity, int32_t n,
                  const vs_fit_params* p, int64_t pair_index0, vs_fit_state* state, double* params, double* affine6,
                  vs_fit_info* info, uint8_t* inliers, void* workspace, size_t ws_bytes, void* stream);

/* fit_motion_noalloc -- for callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc. Same arguments, outputs and errors
 * as vs_fit_motion, without the workspace: the fit kernels use instead a scratch array of
 * VS_FIT_NOALLOC_SCRATCH_BYTES that the library holds in static device memory, one copy per GPU,
 * until the process ends. The call allocates nothing (no hipMalloc, hipFree or allocating library
 * routine). At most vs_fit_noalloc_max_pairs(capacity) pairs per call (the workspace the same call
 * would take from vs_fit_workspace must fit the scratch); a larger n returns VS_ERR_WORKSPACE with
 * nothing enqueued. `stream` must belong to the current device (else VS_ERR_INVALID). Every call on
 * one GPU uses that GPU's one scratch array: calls that may overlap on the device (different streams
 * without ordering between them) race and must be serialised by the caller; calls on one stream are
 * ordered. The scratch needs no clearing: each call writes every byte of it that it reads. The first
 * call on a device looks up that device's scratch address (hipGetSymbolAddress) and keeps it. */
#define VS_FIT_NOALLOC_SCRATCH_BYTES (8 * 1024 * 1024)
int32_t vs_fit_noalloc_max_pairs(int32_t capacity);
int vs_fit_motion_noalloc(const float* src, const float* dst, const uint8_t* valid, int32_t capacity, int32_t n,
                          const vs_fit_params* p, int64_t pair_index0, vs_fit_state* state, double* params,
                          double* affine6, vs_fit_info* info, uint8_t* inliers, void* stream);

/* ---------------------------------------------------------------------------------------------
 * smooth_trajectory -- Section 5.1 (accumulate the per-pair parameters into a trajectory, smooth
 * it with an averaging window of twice the smoothing radius, correct each frame by smoothed minus
 * accumulated) and the sliding parameter store of the real-time version (Section 6).
 * Per pair: (tx, ty, angle = atan2(b, a), log-scale = ln |a + ib|); P_0 = 0, P_j = P_{j-1} + pair_{j-1}.
 * CENTERED: Q_j = mean of P_i, i in [j - r, j + r] clipped to the known sequence; frame j is
 * emitted once P_{j+r} is known or at end of stream, so a stream fed pair by pair emits exactly
 * what one call over the whole sequence emits. CAUSAL: mean over [j - 2r, j]. KALMAN: per
 * parameter random-walk filter, measurement noise 1, process noise kalman_ratio, started at P_0.
 * Correction D_j = Q_j - P_j becomes the matrix mats[k] = Z o T(D_j) (2x3, row-major, maps frame
 * pixel coordinates to output pixel coordinates), T a similarity about (cx, cy), Z a zoom by
 * 1 / (1 - 2 crop) about (cx, cy).
 * pair_params: n_new new pairs [n_new][4] (device). state: one per stream, vs_traj_state_bytes()
 * bytes, initialised by vs_traj_state_init (radius <= 127). Emitted frames go to mats[0..],
 * at most mats_capacity of them; *n_emitted and *first_frame (device) receive the count and the
 * index of the first emitted frame. */
typedef struct {
    int32_t mode;
    int32_t radius;
    double kalman_ratio;
    double crop;
    double cx, cy;
} vs_smooth_params;

size_t vs_traj_state_bytes(void);
int vs_traj_state_init(void* state, void* stream);
int vs_smooth_trajectory(const double* pair_params, int32_t n_new, int32_t end_of_stream, const vs_smooth_params* p,
                         void* state, double* mats, int32_t mats_capacity, int32_t* n_emitted, int64_t* first_frame,
                         void* stream);

/* ---------------------------------------------------------------------------------------------
 * warp_frame -- Section 5 (warp each frame by its corrected transform; cropping is folded into
 * the matrix). Output pixel x takes the bilinear sample of the source at M^-1 x (FP32 coordinates,
 * M inverted in binary64), source samples outside the image take `border`, rounded half up and
 * clamped to [0, 255]. Item i: src + i * src_stride (pitch src_pitch), M = mats + i * mat_stride
 * doubles (6 per matrix), dst + i * dst_stride (pitch dst_pitch); output size = input size. */
int vs_warp_frame(const uint8_t* src, int64_t src_stride, int32_t width, int32_t height, int32_t src_pitch,
                  const double* mats, int64_t mat_stride, uint8_t* dst, int64_t dst_stride, int32_t dst_pitch,
                  int32_t n, int32_t border, void* stream);

/* ---------------------------------------------------------------------------------------------
 * Photometric check and refinement of fitted pair similarities. An extension beyond the six stages
 * above: the brightness constancy of Section 3.2 (Eq. 3) applied to the whole frame under the
 * similarity of Section 4.1 (Eq. 7).
 * Definitions. S(F, p) is the bilinear interpolant of F extended by edge replication; its gradient is
 * the derivative of the bilinear piece in cell floor(p). T_theta(x) = x + [[a, -b], [b, a]] (x - c) / rho
 * + t with theta = (a, b, tx, ty); a fitted similarity (A, B, TX, TY) in centred coordinates
 * (vs_fit_similarity) is theta = (rho (A - 1), rho B, TX, TY) with c = ((W-1)/2, (H-1)/2). The loss of
 * a pair is L = sum over x in the rectangle omega of r(x)^2, r = S(next, T(x)) - prev(x), and
 * J(x) = grad S . dT/dtheta. All arithmetic is binary64.
 * Items: n pairs, pair i reads prev + i * frame_stride, next + i * frame_stride and
 * theta[i * theta_stride + 0..3] (device). omega (host) is shared; 0 <= x0, y0 and x1 <= W, y1 <= H.
 * sums[i * VS_PHOTO_SUMS + k] (device), fully written by the call:
 *   k = 0 the loss; 1..4 dL/dtheta; 5..14 the upper triangle of J^T J row by row
 *   (00 01 02 03 11 12 13 22 23 33); 15..18 J^T r. vs_photometric_fwd fills only k = 0 (the rest 0).
 * Every sum is formed in a fixed order (per-tile partial sums in the workspace, then a per-pair
 * reduction over the tiles in tile order), so repeated calls give bit-identical results.
 * workspace (device, 256-byte aligned): at least vs_photometric_workspace(n, width, height) bytes;
 * no state survives the call.
 */
#define VS_PHOTO_SUMS 19
typedef struct {
    int32_t x0, y0, x1, y1;
} vs_rect;

size_t vs_photometric_workspace(int32_t n, int32_t width, int32_t height);
int vs_photometric_fwd(const uint8_t* prev, const uint8_t* next, int64_t frame_stride, int32_t width, int32_t height,
                       int32_t pitch, int32_t n, const double* theta, int64_t theta_stride, double cx, double cy,
                       double rho, const vs_rect* omega, double* sums, void* workspace, size_t ws_bytes, void* stream);
int vs_photometric_bwd(const uint8_t* prev, const uint8_t* next, int64_t frame_stride, int32_t width, int32_t height,
                       int32_t pitch, int32_t n, const double* theta, int64_t theta_stride, double cx, double cy,
                       double rho, const vs_rect* omega, double* sums, void* workspace, size_t ws_bytes, void* stream);

/* Per-feature window loss (same sampler), the displacement part of the photometric residual of
 * Eq. 3: for point k of pair i (pair i reads prev + i * frame_stride and next + i * frame_stride;
 * its points are u[i * m + k][2] and displacements d[i * m + k][2], float, device),
 * loss[i * m + k] = sum over q in [-win_half, win_half]^2 of (S(next, u + d + q) - S(prev, u + q))^2
 * and grad[i * m + k][2] = dloss/dd (may be NULL). 0 <= win_half <= 31. Each point's sums are
 * reduced in a fixed order (deterministic). */
int vs_photometric_features(const uint8_t* prev, const uint8_t* next, int64_t frame_stride, int32_t width,
                            int32_t height, int32_t pitch, int32_t n, const float* u, const float* d, int32_t m,
                            int32_t win_half, double* loss, double* grad, void* stream);

/* Gauss-Newton refinement of n pairs from theta0: each step solves (J^T J) delta = -J^T r at the
 * current parameters and accepts theta + delta only if the loss decreases; a pair stops at its first
 * rejected step, when J^T J is not positive definite, or after max_steps (0..100) accepted steps.
 * param_kind VS_PHOTO_THETA: theta0/theta_out hold theta; VS_PHOTO_FIT: they hold fitted similarities
 * (A, B, TX, TY) in centred coordinates (converted with the rho given). skip (may be NULL, device):
 * pair i is left unchanged (loss_out 0, accepted 0) when skip[i * skip_stride] != 0; this accepts the
 * `skipped` field of vs_fit_info records (skip = &info[0].skipped, skip_stride = sizeof(vs_fit_info) / 4).
 * Outputs (device): theta_out[i * theta_stride + 0..3] (may alias theta0), loss_out[i][2] = (initial,
 * final) (may be NULL), accepted[i] = accepted steps (may be NULL). workspace: at least
 * vs_photometric_workspace(n, width, height) bytes, 256-byte aligned; no state survives the call.
 * The sums are those of vs_photometric_bwd, so every decision is reproducible. */
#define VS_PHOTO_THETA 0
#define VS_PHOTO_FIT 1
int vs_photometric_refine(const uint8_t* prev, const uint8_t* next, int64_t frame_stride, int32_t width, int32_t height,
                          int32_t pitch, int32_t n, const double* theta0, double* theta_out, int64_t theta_stride,
                          int32_t param_kind, const int32_t* skip, int64_t skip_stride, double cx, double cy, double rho,
                          const vs_rect* omega, int32_t max_steps, double* loss_out, int32_t* accepted, void* workspace,
                          size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------------------------
 * stream_push -- the real-time version of Section 6 on one stream, frame by frame, driven from
 * native code: one call per pushed frame enqueues its pyramid, the tracking of the previous
 * frame's points with the backward check (Sections 3.2, 4.1), the fit with the dwell switch and
 * the skip rule (Section 4), the optional photometric refinement, the re-detection (every
 * redetect_every frames, and on the device after a pair with fewer than min_valid points), the
 * smoother's step with the sliding parameter store (Sections 5.1, 6) and the warps of the frames
 * it emits (Section 5). The result equals the whole-sequence path's, frame for frame. The corners
 * detected on a frame serve only the next pair, so a push enqueues that detection last, after the
 * warps of the frames it emits (and after recording ready_event).
 * The caller sets the geometry, parameters and device buffers below, keeps the struct (host
 * memory) and every buffer alive while the stream runs, and keeps each pushed frame (device,
 * width x height, pitch = width) unchanged until it has been emitted. vs_stream_reset starts a new
 * stream (progress fields, fit and trajectory state). The library allocates nothing and never
 * synchronises the host; all work goes to `stream`. Emitted frames: *first_emitted (host) is the
 * index of the first frame emitted by the call and *n_emitted (host) their count; frame e is
 * complete in out + (e % out_slots) * width * height once the stream reaches the call's end.
 * The smoother's lag is radius for VS_SMOOTH_CENTERED and 0 otherwise; radius <= 127.
 * Errors: VS_ERR_INVALID for a null struct, frame or output, or a bad size; errors of the
 * underlying calls are passed on (work enqueued before a failing launch stays enqueued). */
#define VS_STREAM_MAX_FRAMES 160
typedef struct {
    /* geometry and parameters */
    int32_t width, height;
    vs_pyramid layout;
    vs_detect_params detect;
    vs_lk_params lk;
    vs_fit_params fit;
    vs_smooth_params smooth;
    int32_t capacity;          /* point slots, >= detect.max_corners */
    int32_t redetect_every;
    int32_t min_valid;
    int32_t border;
    int32_t out_slots;         /* output ring length */
    int32_t photo_steps;       /* photometric refinement steps per pair (0: off) */
    vs_rect photo_omega;
    /* device buffers */
    uint8_t* pyr;              /* 2 * layout.bytes */
    float* pts;                /* [2][capacity][2] */
    uint8_t* alive;            /* [2][capacity] */
    float* dst;                /* [capacity][2] */
    uint8_t* status;           /* [capacity] */
    float* fb_err;             /* [capacity] */
    int32_t* n_valid;          /* [1] */
    int32_t* count;            /* [1] */
    void* detect_ws;           /* vs_detect_workspace(width, height, 1) bytes */
    size_t detect_ws_bytes;
    void* fit_ws;              /* vs_fit_workspace(1, capacity) bytes */
    size_t fit_ws_bytes;
    vs_fit_state* fit_state;
    double* pair_params;       /* [1][4], the last pair's (a, b, tx, ty) */
    double* affine6;           /* [1][6], the last pair's 2x3 model */
    vs_fit_info* info;         /* [1] */
    uint8_t* inliers;          /* [capacity] */
    void* traj_state;          /* vs_traj_state_bytes() bytes */
    double* mats;              /* [lag + 2][6] */
    int32_t* n_emitted;        /* [1] */
    int64_t* first_frame;      /* [1] */
    double* photo_loss;        /* [1][2], when photo_steps > 0 */
    int32_t* photo_accepted;   /* [1], when photo_steps > 0 */
    void* photo_ws;            /* vs_photometric_workspace(1, width, height) bytes, when photo_steps > 0 */
    size_t photo_ws_bytes;
    uint8_t* out;              /* [out_slots][height][width] */
    void* ready_event;         /* optional hipEvent_t (NULL: none), recorded on `stream` by every
                                  push once the frames it emits are written, before the re-detection
                                  that only serves the next pair */
    const uint8_t* ring;       /* batched use (vs_batch_push): the stream's frames, frame j at
                                  ring + (j % ring_len) * width * height (16-byte aligned; NULL otherwise) */
    int32_t ring_len;          /* >= lag + 2 when ring is set */
    int32_t ring_pad;
    /* progress, maintained by the library */
    int64_t next_frame;        /* index of the next pushed frame */
    int64_t emitted;           /* frames emitted so far */
    const uint8_t* frames[VS_STREAM_MAX_FRAMES];   /* frame j at [j % (lag + 2)] until emitted */
} vs_stream;

int vs_stream_reset(vs_stream* s, void* stream);
int vs_stream_push(vs_stream* s, const uint8_t* frame, int64_t* first_emitted, int32_t* n_emitted, void* stream);
int vs_stream_flush(vs_stream* s, int64_t* first_emitted, int32_t* n_emitted, void* stream);

/* ---------------------------------------------------------------------------------------------
 * batch_push -- the real-time version of Section 6 for many streams at once: one call processes the
 * next frame of every listed stream of a batch with ONE launch per stage (pyramids, tracking with the
 * backward check, fits with the dwell switch and skip rule, the smoother's step, the warps of the
 * emitted frames, the re-detections), the stages and their order being those of vs_stream_push. Every
 * stream's outputs are those vs_stream_push gives on the same frames, bit for bit.
 * A batch is one class of streams: same geometry, capacity and parameters except the corner budget
 * (detect.max_corners), the RANSAC seed and the stream id (fit.seed, fit.stream_id), which are per
 * stream. The prototype given to vs_batch_init fixes the class; photometric refinement is not part of
 * the batched step (photo_steps must be 0).
 * Each stream keeps its own vs_stream struct and device buffers (as for vs_stream_push, plus a frame
 * ring: frame j must be at ring + (j % ring_len) * width * height when the push that processes it
 * runs, and stay there until emitted). vs_batch_attach resets the stream (frame 0 next) and records
 * its buffers in a device descriptor in the batch workspace; from then on the stream advances only
 * through vs_batch_push until vs_batch_detach; vs_stream_flush ends it as usual (its state is the
 * single-stream one).
 * vs_batch_push(b, n, slots, first_emitted, n_emitted, stream): items are the n distinct attached
 * slots (host array); first_emitted[k] / n_emitted[k] (host) receive the index and count (0 or 1) of
 * the frames item k emits: frame e is in out + (e % out_slots) * width * height once the stream reaches
 * the call's end (and ready_event, when set, is recorded after the warps, before the re-detections).
 * The device work depends only on the slots (each stream's frame counter is kept on the device), so a
 * push over a fixed slot list may be captured in a graph and replayed once per frame: the capture
 * advances the host progress once; after k replays call vs_batch_note_replayed(b, n, slots, k - 1).
 * workspace (device, 256-byte aligned): vs_batch_workspace(proto, max_streams, detect_chunk) bytes:
 * descriptors, the step's slot list, the fit workspace of max_streams pairs and the detection
 * workspace of detect_chunk frames (the detection runs in chunks of that many items).
 * Errors: VS_ERR_INVALID for a bad slot, a slot listed twice, a stream of another class, a missing or
 * misaligned ring or pyramid; nothing is enqueued then. */
#define VS_BATCH_MAX_STREAMS 256
typedef struct {
    vs_stream proto;           /* the class: geometry and shared parameters (copied by vs_batch_init) */
    int32_t max_streams;       /* descriptor slots, <= VS_BATCH_MAX_STREAMS */
    int32_t detect_chunk;      /* items per detection launch */
    void* workspace;           /* device */
    size_t ws_bytes;
    void* ready_event;         /* optional hipEvent_t recorded after each push's warps (NULL: none) */
    vs_stream* attached[VS_BATCH_MAX_STREAMS];   /* host: the stream of each slot (NULL: free) */
} vs_batch;

size_t vs_batch_workspace(const vs_stream* proto, int32_t max_streams, int32_t detect_chunk);
int vs_batch_init(vs_batch* b, const vs_stream* proto, int32_t max_streams, int32_t detect_chunk, void* workspace,
                  size_t ws_bytes);
int vs_batch_attach(vs_batch* b, int32_t slot, vs_stream* s, void* stream);
int vs_batch_detach(vs_batch* b, int32_t slot);
int vs_batch_push(vs_batch* b, int32_t n, const int32_t* slots, int64_t* first_emitted, int32_t* n_emitted,
                  void* stream);
int vs_batch_note_replayed(vs_batch* b, int32_t n, const int32_t* slots, int32_t steps);

/* ---------------------------------------------------------------------------------------------
 * tuning -- launch-shape choices that change speed only, never a result bit (the choices only
 * reorder independent workgroups, group independent waves, or split independent work differently).
 * Process-wide; a call reads the values current when it is made, so settings may change between
 * calls from any thread.
 *   xcd_min_items_{pyramid,lk,warp}: batches of at least this many items keep each item's
 *     workgroups on one XCD (one L2); 0 selects the default (8); 1 always, 65536 never.
 *   lk_points_per_group: points (one wave each) per tracking workgroup, 1, 2 or 4; 0: default (1).
 *   detect_segment_rows: output rows per wave segment of the corner response, 12..240; 0: by batch
 *     size (12 for at most 8 frames, else 60). Candidates are sorted afterwards, so the split is free.
 *   fit_groups_in_flight: hypothesis workgroups of a fit launch are spread until about this many are
 *     in flight (at most 32 per pair), 64..16384; 0: default (2048). The best hypothesis is the most
 *     inliers, then the smallest index, whatever the split.
 * vs_set_tuning(NULL) restores the defaults. Values out of range: VS_ERR_INVALID, nothing changed.
 * vs_get_tuning reports the values in force (defaults resolved; detect_segment_rows 0 = by batch
 * size). Both are host-only. */
typedef struct {
    int32_t xcd_min_items_pyramid;
    int32_t xcd_min_items_lk;
    int32_t xcd_min_items_warp;
    int32_t lk_points_per_group;
    int32_t detect_segment_rows;
    int32_t fit_groups_in_flight;
} vs_tuning;

int vs_set_tuning(const vs_tuning* t);
int vs_get_tuning(vs_tuning* t);

/* ---------------------------------------------------------------------------------------------
 * misc */
const char* vs_last_error(void);   /* thread-local message of the last failing call */
int vs_version(void);

#ifdef __cplusplus
}
#endif
#endif /* VSTAB_H */
