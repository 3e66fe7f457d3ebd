// smooth_trajectory: per-stream trajectory accumulation, smoothing and correction matrices.
//
// One 256-thread workgroup per call. Thread 0 appends the new pairs to the trajectory in order
// (binary64, sequential, as the definition states) into a ring of the last VS_TRAJ_RING frame
// positions kept in the caller's device state; then every thread emits frames whose smoothing
// window is complete, summing the window directly in ascending frame order. Because each
// emitted value depends only on the positions (not on how the pairs were split across calls),
// feeding a stream pair by pair emits bit-for-bit what one call over the whole sequence emits.
// Long calls are processed in chunks small enough for the ring.
#include <cmath>

#include "vs_common.hpp"

#pragma clang fp contract(off)

namespace {

struct TrajState {
    int64_t known;      // frames whose position P_j is known (P_0 = 0 at start)
    int64_t emitted;    // frames emitted so far
    double kx[4];       // Kalman estimate
    double kS[4];       // Kalman posterior variance
    double ring[VS_TRAJ_RING][4];   // P_j at j % VS_TRAJ_RING
    double kq[VS_TRAJ_RING][4];     // Kalman output Q_j at j % VS_TRAJ_RING
};

__global__ void traj_init_kernel(TrajState* s)
{
    const int t = threadIdx.x;
    if (t == 0) {
        s->known = 1;
        s->emitted = 0;
        for (int c = 0; c < 4; ++c) {
            s->kx[c] = 0.0;
            s->kS[c] = 0.0;
        }
    }
    for (int i = t; i < VS_TRAJ_RING * 4; i += blockDim.x) {
        (&s->ring[0][0])[i] = 0.0;
        (&s->kq[0][0])[i] = 0.0;
    }
}

struct SmoothArgs {
    int mode, radius;
    double ratio, crop, cx, cy;
};

__device__ void emit_frame(const double (*ring)[4], const double (*kq)[4], const SmoothArgs& a, int64_t j,
                           int64_t last_known, double* M)
{
    double q[4];
    const double* P = ring[j % VS_TRAJ_RING];
    if (a.mode == VS_SMOOTH_KALMAN) {
        for (int c = 0; c < 4; ++c) q[c] = kq[j % VS_TRAJ_RING][c];
    } else {
        const int64_t lo = (a.mode == VS_SMOOTH_CENTERED) ? (j - a.radius > 0 ? j - a.radius : 0)
                                                          : (j - 2 * a.radius > 0 ? j - 2 * a.radius : 0);
        int64_t hi = (a.mode == VS_SMOOTH_CENTERED) ? j + a.radius : j;
        hi = hi < last_known ? hi : last_known;
        for (int c = 0; c < 4; ++c) {
            double sum = 0.0;
            for (int64_t i = lo; i <= hi; ++i) sum += ring[i % VS_TRAJ_RING][c];
            q[c] = sum / (double)(hi - lo + 1);
        }
    }
    const double dx = q[0] - P[0], dy = q[1] - P[1], da = q[2] - P[2], ds = q[3] - P[3];
    const double z = 1.0 / (1.0 - 2.0 * a.crop);
    const double sc = exp(ds);
    const double ca = sc * cos(da), sb = sc * sin(da);
    M[0] = z * ca;
    M[1] = -z * sb;
    M[2] = z * (dx - ca * a.cx + sb * a.cy) + a.cx;
    M[3] = z * sb;
    M[4] = z * ca;
    M[5] = z * (dy - sb * a.cx - ca * a.cy) + a.cy;
}

// What one smoothing item reads and writes.
struct SmoothItem {
    const double* pairs;
    int n_new;
    TrajState* s;
    double* mats;
    int32_t* n_emitted;
    int64_t* first_frame;
};

// the one stream of a vs_smooth_trajectory call
struct Single {
    SmoothItem it;
    __device__ __forceinline__ SmoothItem at(int) const { return it; }
};

// item i of a batched step: the stream's pair j - 1 (none at j = 0)
struct Step {
    vs::StepView v;
    __device__ __forceinline__ SmoothItem at(int i) const
    {
        const vs::StepStream& d = v.s(i);
        return SmoothItem{d.pair_params, d.next_frame > 0 ? 1 : 0, static_cast<TrajState*>(d.traj_state), d.mats,
                          d.n_emitted, d.first_frame};
    }
};

// one workgroup per item (blockIdx.x)
template <class IO>
__global__ __launch_bounds__(256) void smooth_kernel(IO io, int eos, SmoothArgs a, int mats_cap)
{
    const SmoothItem item = io.at(blockIdx.x);
    const double* __restrict__ pairs = item.pairs;
    const int n_new = item.n_new;
    TrajState* s = item.s;
    double* __restrict__ mats = item.mats;
    int32_t* n_emitted = item.n_emitted;
    int64_t* first_frame = item.first_frame;
    // the ring (and Kalman outputs) live in LDS during the call; the per-pair parameter
    // conversions run in parallel, only the 4 running sums are sequential (one thread each)
    __shared__ double ring[VS_TRAJ_RING][4];
    __shared__ double kq[VS_TRAJ_RING][4];
    __shared__ double dlt[VS_TRAJ_RING][4];
    __shared__ int64_t s_known, s_emitted, s_first;
    __shared__ int s_count;
    const int t = threadIdx.x;
    const int window = (a.mode == VS_SMOOTH_KALMAN) ? 0 : 2 * a.radius;
    const int chunk = VS_TRAJ_RING - window - 1;
    for (int i = t; i < VS_TRAJ_RING * 4; i += 256) {
        (&ring[0][0])[i] = (&s->ring[0][0])[i];
        (&kq[0][0])[i] = (&s->kq[0][0])[i];
    }
    double kx = 0.0, kS = 0.0;
    if (t < 4) {
        kx = s->kx[t];
        kS = s->kS[t];
    }
    if (t == 0) {
        s_known = s->known;
        s_emitted = s->emitted;
        s_first = s->emitted;
        s_count = 0;
    }
    __syncthreads();
    int consumed = 0;
    while (true) {
        const int take = (n_new - consumed) < chunk ? (n_new - consumed) : chunk;
        for (int k = t; k < take; k += 256) {
            const double* q = pairs + 4 * (int64_t)(consumed + k);
            dlt[k][0] = q[2];
            dlt[k][1] = q[3];
            dlt[k][2] = atan2(q[1], q[0]);
            dlt[k][3] = log(sqrt(q[0] * q[0] + q[1] * q[1]));
        }
        __syncthreads();
        const int64_t known0 = s_known;
        if (t < 4) {
            // P_j = P_{j-1} + d_{j-1} for parameter t, in order
            double p = ring[(known0 - 1) % VS_TRAJ_RING][t];
            for (int k = 0; k < take; ++k) {
                const int64_t j = known0 + k;
                p = p + dlt[k][t];
                ring[j % VS_TRAJ_RING][t] = p;
                if (a.mode == VS_SMOOTH_KALMAN) {
                    const double Sm = kS + a.ratio;
                    const double K = Sm / (Sm + 1.0);
                    kx = kx + K * (p - kx);
                    kS = (1.0 - K) * Sm;
                    kq[j % VS_TRAJ_RING][t] = kx;
                }
            }
        }
        consumed += take;
        __syncthreads();
        const bool last = consumed >= n_new;
        const int64_t known = known0 + take;
        int64_t end;     // frames [s_emitted, end) are emitted now
        if (a.mode == VS_SMOOTH_CENTERED) end = (last && eos) ? known : known - a.radius;
        else end = known;
        if (end < s_emitted) end = s_emitted;
        const int64_t e0 = s_emitted;
        for (int64_t j = e0 + t; j < end; j += 256) {
            const int64_t k = j - s_first;
            if (k < mats_cap) emit_frame(ring, kq, a, j, known - 1, mats + 6 * k);
        }
        __syncthreads();
        if (t == 0) {
            s_known = known;
            s_count += (int)(end - e0);
            s_emitted = end;
        }
        __syncthreads();
        if (last) break;
    }
    for (int i = t; i < VS_TRAJ_RING * 4; i += 256) {
        (&s->ring[0][0])[i] = (&ring[0][0])[i];
        (&s->kq[0][0])[i] = (&kq[0][0])[i];
    }
    if (t < 4) {
        s->kx[t] = kx;
        s->kS[t] = kS;
    }
    if (t == 0) {
        s->known = s_known;
        s->emitted = s_emitted;
        if (n_emitted) *n_emitted = s_count < mats_cap ? s_count : mats_cap;
        if (first_frame) *first_frame = s_first;
    }
}

SmoothArgs smooth_args(const vs_smooth_params& p)
{
    SmoothArgs a;
    a.mode = p.mode;
    a.radius = p.radius;
    a.ratio = p.kalman_ratio;
    a.crop = p.crop;
    a.cx = p.cx;
    a.cy = p.cy;
    return a;
}

int check_smooth(const vs_smooth_params& p)
{
    if (p.mode < VS_SMOOTH_CENTERED || p.mode > VS_SMOOTH_KALMAN)
        return vs::set_error(VS_ERR_INVALID, "vs_smooth_trajectory: bad mode");
    if (p.mode != VS_SMOOTH_KALMAN && (p.radius < 0 || 2 * p.radius + 2 > VS_TRAJ_RING))
        return vs::set_error(VS_ERR_UNSUPPORTED, "vs_smooth_trajectory: radius must be 0..%d", (VS_TRAJ_RING - 2) / 2);
    if (p.mode == VS_SMOOTH_KALMAN && !(p.kalman_ratio > 0.0))
        return vs::set_error(VS_ERR_INVALID, "vs_smooth_trajectory: kalman_ratio must be > 0");
    if (!(p.crop >= 0.0 && p.crop < 0.5)) return vs::set_error(VS_ERR_INVALID, "vs_smooth_trajectory: crop in [0, 0.5)");
    return VS_OK;
}

}  // namespace

extern "C" size_t vs_traj_state_bytes(void) { return sizeof(TrajState); }

extern "C" int vs_traj_state_init(void* state, void* stream)
{
    if (!state) return vs::set_error(VS_ERR_INVALID, "vs_traj_state_init: null state");
    if (reinterpret_cast<uintptr_t>(state) & 7) return vs::set_error(VS_ERR_INVALID, "vs_traj_state_init: misaligned state");
    traj_init_kernel<<<1, 256, 0, vs::as_stream(stream)>>>(static_cast<TrajState*>(state));
    return vs::check_launch("vs_traj_state_init");
}

extern "C" int vs_smooth_trajectory(const double* pair_params, int32_t n_new, int32_t end_of_stream,
                                    const vs_smooth_params* p, void* state, double* mats, int32_t mats_capacity,
                                    int32_t* n_emitted, int64_t* first_frame, void* stream)
{
    if (!p || !state) return vs::set_error(VS_ERR_INVALID, "vs_smooth_trajectory: null argument");
    if (n_new < 0 || mats_capacity < 0 || (n_new > 0 && !pair_params) || (mats_capacity > 0 && !mats))
        return vs::set_error(VS_ERR_INVALID, "vs_smooth_trajectory: bad counts");
    const int e = check_smooth(*p);
    if (e) return e;
    const Single io{SmoothItem{pair_params, n_new, static_cast<TrajState*>(state), mats, n_emitted, first_frame}};
    smooth_kernel<<<1, 256, 0, vs::as_stream(stream)>>>(io, end_of_stream, smooth_args(*p), mats_capacity);
    return vs::check_launch("vs_smooth_trajectory");
}

namespace vs {

// the smoother's step of every item of a batched step: the pair j - 1 (j > 0) appended, the frames it
// completes emitted to the stream's mats
int step_smooth(const StepView& v, int n, const vs_smooth_params& p, hipStream_t s)
{
    if (n <= 0) return VS_OK;
    const int e = check_smooth(p);
    if (e) return e;
    smooth_kernel<<<n, 256, 0, s>>>(Step{v}, 0, smooth_args(p), v.lag + 2);
    return check_launch("vs_batch_push(smooth)");
}

}  // namespace vs
