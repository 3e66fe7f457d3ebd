// track_lk: pyramidal Lucas-Kanade with the forward-backward check, one wave64 per point slot.
//
// Lane layout for a (2h+1)^2 window: the window's 2h+1 columns are spread over the lanes and the
// rows over G = 64 / (2h+1) lane groups, each group owning R = ceil((2h+1) / G) consecutive rows
// (h = 10: 21 columns x 3 groups of 7 rows = 63 lanes). Lanes outside every group read zeros (an
// out-of-range buffer offset, or a zeroed LDS area), so all their terms vanish; when the window's
// rows do not fill every group's R rows, the samples past the window get zero gradient weight.
// Every lane runs the same branch-free loops. All samples of a window share one fractional offset,
// so per level a lane reads its (R+3) x 4 previous-frame block once, interpolates each row
// horizontally first and derives I and the two central differences of its R samples into
// registers. When the whole window is inside the level and R <= 7, the window's block (24 rows of
// 32 bytes) is staged in the wave's LDS by one 16-byte load per lane pair and each lane reads its
// rows there as two aligned words; a wave64 buffer load occupies the texture address unit for
// about the same time whatever its width, so this replaces 10 row loads per set-up. Larger windows
// load one unaligned 32-bit word per row; windows at the level's edge take edge-clamped byte loads.
// The differences are kept without their factor 1/2 (D = 2 grad I): the tensor then carries a
// factor 4 and the residual sums a factor 2, both exact powers of two, which the minimum-eigenvalue
// test and the step solve absorb.
//
// Gauss-Newton iterations: all samples also share the iterate's fractional offset (ja, jb), so the
// residual sum over the window, sum (I - J) grad I, is E0 - ja E1 - jb E2 - ja jb E3 with four sums
// per gradient component that depend only on the iterate's integer position (the bilinear form of
// the next-frame 2 x 2 blocks; see residual_partials). They are recomputed, from the lane's (R+1) x 2
// next-frame block (staged like the previous-frame block), only when the integer position moves;
// an iteration that stays on the same pixel costs a few wave-uniform operations. The lanes
// accumulate plain sums of products of raw next-frame pixels with the gradients (no per-sample
// differences), and the E sums are formed from the totals. The first block of each level is read
// with the set-up, and its eight sums share the set-up's reduction with the three tensor sums and
// the two sums of I times the gradient. The sums are reduced through LDS (a transposed store,
// chunk sums, totals read back by every lane), which costs only additions on the vector ALU; the
// iteration control is wave-uniform. One wave per point lets every point retire independently.
#include "vs_common.hpp"

namespace {

constexpr uint32_t RSRC_WORD3 = 0x00020000;   // raw (untyped) buffer access on gfx9-family parts
// vector offset of lanes outside the window: at or past 2^31, beyond every level's byte count (the
// host limits a level to fewer than 2^31 bytes), so their buffer loads return 0
constexpr int OOB = -2147483647 - 1;

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
    int full;          // the window's rows fill every lane group's `rows` rows exactly
    float eps2, eig_thr;   // eig_thr = 4 N min_eig
};

__device__ __forceinline__ bool wave_all(bool c) { return __ballot(!c) == 0; }
// a value every lane holds equally, kept in a scalar register (frees a vector register while it waits)
__device__ __forceinline__ float wave_uniform(float x)
{
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}
// for a condition every lane evaluates identically: a scalar branch condition
__device__ __forceinline__ bool uniform(bool c) { return __ballot(c) != 0; }

// Per-wave LDS scratch of the window sums: 64 chunk sums and 16 totals first (within reach of the
// LDS instructions' immediate offsets from the area's base), then the lanes' values stored
// transposed (value j of lane l at RED_T + j * RED_STRIDE + l; the odd stride puts the lanes of
// every later read on distinct banks).
constexpr int RED_STRIDE = 65;
constexpr int RED_T = 64 + 16;
constexpr int RED_FLOATS = RED_T + 16 * RED_STRIDE;
// The same per-wave area first holds staged image blocks: STAGE_ROWS rows of 32 bytes (the window's
// rows, 4-byte aligned at the left), written by one 16-byte load per lane pair. A zeroed area after
// it serves the lanes outside the window, whose reads must return 0.
constexpr int STAGE_ROWS = 24;
constexpr int ZERO_FLOATS = 80;   // 10 rows of 32 bytes
constexpr int WAVE_LDS_FLOATS = RED_FLOATS + ZERO_FLOATS;
static_assert(STAGE_ROWS * 8 <= RED_FLOATS && WAVE_LDS_FLOATS % 4 == 0, "staging fits the reduction area");

using vs::wave_lds_sync;

// Wave totals of the first M of N (8 or 16) values per lane, returned in every lane. Lane l adds value
// l % N over the N lanes of its chunk l / N, lane j < M then adds the 64 / N chunk sums of value j, and
// every lane reads the M totals back (a broadcast read). The order of the additions is fixed, so the
// totals are the same in every lane and on every run. The cross-lane traffic goes through LDS, which
// costs no vector ALU cycles beyond the additions.
template <int N, int M>
__device__ __forceinline__ void wave_sums(const float (&v)[N], float (&tot)[M], float* red)
{
    static_assert(N == 8 || N == 16, "8 or 16 values per lane");
    constexpr int C = 64 / N;   // chunks
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int j = 0; j < M; ++j) red[RED_T + j * RED_STRIDE + lane] = v[j];
    wave_lds_sync();
    const int vj = lane % N, ch = lane / N;
    const float* col = red + RED_T + vj * RED_STRIDE + ch * N;
    float s = col[0];
#pragma unroll
    for (int i = 1; i < N; ++i) s += col[i];
    float* part = red;
    part[vj * C + ch] = s;
    wave_lds_sync();
    float* T = part + 64;
    if (lane < M) {
        float t = part[lane * C];
#pragma unroll
        for (int k = 1; k < C; ++k) t += part[lane * C + k];
        T[lane] = t;
    }
    wave_lds_sync();
#pragma unroll
    for (int j = 0; j < M; ++j) tot[j] = T[j];
    wave_lds_sync();   // the next call's stores come after these reads
}

// Stages rows r0 .. r0 + nr - 1, bytes c0 .. c0 + 31 (c0 a multiple of 4) of the level into the wave's
// LDS rows (32 bytes each): lane 2r + h loads row r's 16-byte half h with one load. Bytes past the
// level's range read as 0 (buffer range check); the caller uses only bytes inside the level.
__device__ __forceinline__ void stage_rows(const Img& A, int r0, int nr, int c0, uint32_t* rows)
{
    const int lane = threadIdx.x & 63;
    const int r = lane >> 1, h = lane & 1;
    if (r < nr) {
        const int off = (int)__umul24((unsigned)(r0 + r), (unsigned)A.pitch) + c0 + 16 * h;
        typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
        const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(A.rs, off, 0, 0);
        *reinterpret_cast<u32x4*>(rows + 8 * r + 4 * h) = v;
    }
    wave_lds_sync();
}

// the 4 bytes at byte offset 4 * word + shift of an LDS area (shift 0..3), read as two aligned words
__device__ __forceinline__ uint32_t lds_word(const uint32_t* p, unsigned shift)
{
    return __builtin_amdgcn_alignbyte(p[1], p[0], shift);
}

// Next-frame 2-pixel rows x0, x0 + 1 of rows y0 .. y0 + RMAX: qa = P(x0), qb = P(x0 + 1). The lane's
// block sits at column gcol and row lrow of the window's block, whose origin is (bx, by). When every
// active lane's block is inside the level: for windows of at most 7 rows per lane the window's
// 22-row block is staged in LDS with one load and each lane reads its rows there; larger windows
// load one (unaligned) 16-bit word per row, the row offset in the load's scalar offset. Otherwise
// edge-clamped byte loads. Inactive lanes read zeros.
template <int RMAX>
__device__ __forceinline__ void load_next_block(const Img& B, int x0, int y0, int bx, int by, int lane_off, bool active,
                                                uint32_t* stage, float (&qa)[RMAX + 1], float (&qb)[RMAX + 1])
{
    const bool b_in = wave_all(!active || (x0 >= 0 && x0 + 1 <= B.w - 1 && y0 >= 0 && y0 + RMAX <= B.h - 1));
    if (b_in) {
        if constexpr (RMAX <= 7) {
            const int c0 = bx & ~3;
            stage_rows(B, by, STAGE_ROWS - 2, c0, stage);
            const int o = active ? lane_off + (bx - c0) : 4 * RED_FLOATS;
            const uint32_t* p = stage + (o >> 2);
            const unsigned sh = (unsigned)(o & 3);
#pragma unroll
            for (int k = 0; k <= RMAX; ++k) {
                const uint32_t w = lds_word(p + 8 * k, sh);
                qa[k] = (float)(w & 0xff);
                qb[k] = (float)((w >> 8) & 0xff);
            }
            wave_lds_sync();   // the area is written again by the next staging or reduction
        } else {
            const int v0 = active ? (int)__umul24((unsigned)y0, (unsigned)B.pitch) + x0 : OOB;
#pragma unroll
            for (int k = 0; k <= RMAX; ++k) {
                const uint32_t w = __builtin_amdgcn_raw_buffer_load_b16(B.rs, v0, k * B.pitch, 0);
                qa[k] = (float)(w & 0xff);
                qb[k] = (float)((w >> 8) & 0xff);
            }
        }
    } else {
        const int c0 = active ? vs::clampi(x0, 0, B.w - 1) : OOB;
        const int c1 = active ? vs::clampi(x0 + 1, 0, B.w - 1) : OOB;
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

// The compiler would turn differences of converted bytes back into integer differences followed by
// conversions; an empty asm statement hides the conversion's origin.
__device__ __forceinline__ float byte_f(uint32_t p)
{
    float f = (float)p;
    asm("" : "+v"(f));
    return f;
}

// Horizontal terms of one previous-frame row from its pixels p0..p3 at columns ix-1 .. ix+2:
// H = P(ix + a) and, with DIFF, D = P(ix + 1 + a) - P(ix - 1 + a) = (p2 - p0) + a ((p3 - p1) - (p2 - p0)).
// The pixel differences are exact in binary32, so each term rounds once. Bytes are converted first
// and differenced as floats: a float subtraction issues at twice the rate of an integer difference
// followed by a conversion.

template <bool DIFF>
__device__ __forceinline__ void row_terms(uint32_t p0, uint32_t p1, uint32_t p2, uint32_t p3, float a, float& H, float& D)
{
    const float f1 = byte_f(p1), f2 = byte_f(p2);
    H = fmaf(a, f2 - f1, f1);
    if constexpr (DIFF) {
        const float d20 = f2 - byte_f(p0);
        D = fmaf(a, (byte_f(p3) - f1) - d20, d20);
    }
}

// Previous-frame samples of one lane at rows iy .. iy + RMAX - 1 and column ix, offset by the shared
// fraction (a, b): I, Dx = I(x + 1) - I(x - 1) and Dy = I(y + 1) - I(y - 1). Rows iy-1 .. iy+RMAX+1
// and columns ix-1 .. ix+2 are read. With FAST (every lane's block inside the level) and at most 7
// rows per lane, the window's 24-row block (origin (bx, by), 4-byte aligned left edge) is staged in
// LDS with one load and the lane's rows start at byte lane_off of it; with FAST and larger windows,
// one unaligned 32-bit load per row; otherwise four edge-clamped byte loads. Rows are interpolated
// horizontally first; V(r) = lerp(H(r), H(r+1), b) gives I = V(k+1) and Dy = V(k+2) - V(k), and Dx
// interpolates the rows' D vertically. With WEIGHTED, rows k >= nrows get Dx = Dy = 0.
// I, Ix, Iy of one lane from rows held as words at sp (row r at sp + 8 r, the lane's 4 bytes at byte
// shift sh of two aligned words), with the shared fraction (a, b); see window_samples.
template <int RMAX, bool WEIGHTED>
__device__ __forceinline__ void staged_terms(const uint32_t* sp, unsigned sh, float a, float b, int nrows,
                                             float (&I)[RMAX], float (&Ix)[RMAX], float (&Iy)[RMAX])
{
    float H[RMAX + 3], D[RMAX + 3];   // D is used for rows 1 .. RMAX + 1 only
#pragma unroll
    for (int r = 0; r < RMAX + 3; ++r) {
        const uint32_t w = lds_word(sp + 8 * r, sh);
        const uint32_t p0 = w & 0xff, p1 = (w >> 8) & 0xff, p2 = (w >> 16) & 0xff, p3 = w >> 24;
        if (r == 0 || r == RMAX + 2)
            row_terms<false>(p0, p1, p2, p3, a, H[r], D[r]);
        else
            row_terms<true>(p0, p1, p2, p3, a, H[r], D[r]);
    }
    float V[RMAX + 2];
#pragma unroll
    for (int r = 0; r < RMAX + 2; ++r) V[r] = lerp(H[r], H[r + 1], b);
#pragma unroll
    for (int k = 0; k < RMAX; ++k) {
        I[k] = V[k + 1];
        Ix[k] = lerp(D[k + 1], D[k + 2], b);
        Iy[k] = V[k + 2] - V[k];
        if constexpr (WEIGHTED) {
            const float wgt = k < nrows ? 1.0f : 0.0f;
            Ix[k] *= wgt;
            Iy[k] *= wgt;
        }
    }
}

template <int RMAX, bool FAST, bool WEIGHTED>
__device__ __forceinline__ void window_samples(const Img& A, int ix, int iy, int bx, int by, int lane_off, float a,
                                               float b, int nrows, bool active, uint32_t* stage, float (&I)[RMAX],
                                               float (&Ix)[RMAX], float (&Iy)[RMAX])
{
    constexpr bool STAGED = FAST && RMAX <= 7;   // the window's 24-row block staged in LDS
    float H[RMAX + 3], D[RMAX + 3];   // D is used for rows 1 .. RMAX + 1 only
    int v0 = 0;
    const uint32_t* sp = stage;
    unsigned sh = 0;
    if constexpr (STAGED) {
        const int c0 = bx & ~3;
        stage_rows(A, by, STAGE_ROWS, c0, stage);
        const int o = active ? lane_off + (bx - c0) : 4 * RED_FLOATS;
        sp = stage + (o >> 2);
        sh = (unsigned)(o & 3);
    } else {
        v0 = active ? (int)__umul24((unsigned)(iy - 1), (unsigned)A.pitch) + ix - 1 : OOB;
    }
    int c[4];
    if constexpr (!FAST) {
#pragma unroll
        for (int j = 0; j < 4; ++j) c[j] = active ? vs::clampi(ix - 1 + j, 0, A.w - 1) : OOB;
    }
#pragma unroll
    for (int r = 0; r < RMAX + 3; ++r) {
        uint32_t p0, p1, p2, p3;
        if constexpr (FAST) {
            uint32_t w;
            if constexpr (STAGED)
                w = lds_word(sp + 8 * r, sh);
            else
                w = __builtin_amdgcn_raw_buffer_load_b32(A.rs, v0, r * A.pitch, 0);
            p0 = w & 0xff;
            p1 = (w >> 8) & 0xff;
            p2 = (w >> 16) & 0xff;
            p3 = w >> 24;
        } else {
            const int base = (int)__umul24((unsigned)vs::clampi(iy - 1 + r, 0, A.h - 1), (unsigned)A.pitch);
            p0 = __builtin_amdgcn_raw_buffer_load_b8(A.rs, base + c[0], 0, 0);
            p1 = __builtin_amdgcn_raw_buffer_load_b8(A.rs, base + c[1], 0, 0);
            p2 = __builtin_amdgcn_raw_buffer_load_b8(A.rs, base + c[2], 0, 0);
            p3 = __builtin_amdgcn_raw_buffer_load_b8(A.rs, base + c[3], 0, 0);
        }
        if (r == 0 || r == RMAX + 2)
            row_terms<false>(p0, p1, p2, p3, a, H[r], D[r]);
        else
            row_terms<true>(p0, p1, p2, p3, a, H[r], D[r]);
    }
    float V[RMAX + 2];
#pragma unroll
    for (int r = 0; r < RMAX + 2; ++r) V[r] = lerp(H[r], H[r + 1], b);
    if constexpr (STAGED) wave_lds_sync();   // the area is written again by the next staging
#pragma unroll
    for (int k = 0; k < RMAX; ++k) {
        I[k] = V[k + 1];
        Ix[k] = lerp(D[k + 1], D[k + 2], b);
        Iy[k] = V[k + 2] - V[k];
        if constexpr (WEIGHTED) {
            const float wgt = k < nrows ? 1.0f : 0.0f;
            Ix[k] *= wgt;
            Iy[k] *= wgt;
        }
    }
}

// The set-up's two blocks when both lie inside their levels and a lane holds at most 7 rows: the
// previous-frame window block (24 rows) and the first iterate's next-frame block (22 rows) are loaded
// together, so the two global-memory latencies overlap, and staged in two areas of the wave's LDS;
// the previous-frame block's arithmetic runs while the next-frame block is still arriving. Both are
// read as in window_samples and load_next_block (same arithmetic, same results).
template <int RMAX, bool WEIGHTED>
__device__ __forceinline__ void setup_staged(const Img& A, const Img& B, int bx, int by, int nbx, int nby,
                                             int lane_off, float a, float b, int nrows, bool active, float* red,
                                             float (&I)[RMAX], float (&Ix)[RMAX], float (&Iy)[RMAX],
                                             float (&qa)[RMAX + 1], float (&qb)[RMAX + 1])
{
    static_assert(RMAX <= 7, "staged blocks hold 7 rows per lane at most");
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    const int lane = threadIdx.x & 63;
    const int r = lane >> 1, h = lane & 1;
    uint32_t* sprev = reinterpret_cast<uint32_t*>(red);
    uint32_t* snext = sprev + 8 * STAGE_ROWS;
    static_assert(8 * (2 * STAGE_ROWS - 2) <= RED_FLOATS, "both blocks fit the reduction area");
    const int pc0 = bx & ~3, nc0 = nbx & ~3;
    u32x4 vp = {0u, 0u, 0u, 0u}, vn = {0u, 0u, 0u, 0u};
    if (r < STAGE_ROWS)
        vp = __builtin_amdgcn_raw_buffer_load_b128(A.rs, (int)__umul24((unsigned)(by + r), (unsigned)A.pitch) + pc0 + 16 * h,
                                                   0, 0);
    if (r < STAGE_ROWS - 2)
        vn = __builtin_amdgcn_raw_buffer_load_b128(B.rs, (int)__umul24((unsigned)(nby + r), (unsigned)B.pitch) + nc0 + 16 * h,
                                                   0, 0);
    // the previous-frame block first: its arithmetic overlaps the next-frame block's load
    if (r < STAGE_ROWS) *reinterpret_cast<u32x4*>(sprev + 8 * r + 4 * h) = vp;
    wave_lds_sync();
    // lanes outside the window read the zeroed area
    const uint32_t* zero = reinterpret_cast<const uint32_t*>(red + RED_FLOATS);
    const int op = lane_off + (bx - pc0), on = lane_off + (nbx - nc0);
    staged_terms<RMAX, WEIGHTED>(active ? sprev + (op >> 2) : zero, active ? (unsigned)(op & 3) : 0u, a, b, nrows, I, Ix,
                                 Iy);
    if (r < STAGE_ROWS - 2) *reinterpret_cast<u32x4*>(snext + 8 * r + 4 * h) = vn;
    wave_lds_sync();
    const uint32_t* np = active ? snext + (on >> 2) : zero;
    const unsigned nsh = active ? (unsigned)(on & 3) : 0u;
#pragma unroll
    for (int k = 0; k <= RMAX; ++k) {
        const uint32_t w = lds_word(np + 8 * k, nsh);
        qa[k] = (float)(w & 0xff);
        qb[k] = (float)((w >> 8) & 0xff);
    }
    wave_lds_sync();   // the area is written again by the next staging or reduction
}

// The tracks of one point u of frame A into the target frames t0 .. nt - 1 (at most NT; target t is
// frame and pyramid (fb[t], pb[t])). Per level the window set-up over A (samples, gradients, the
// tensor, its eigenvalue test and the sums of I times the gradient) is formed once and serves every
// target; the first target's first next-frame block is read and summed with it, and every later
// target reads its first block as a reload. Each target then runs its own Gauss-Newton iterations
// from its own guess. The arithmetic of a target is that of a track of its own, so its result does
// not depend on the other targets. ok[t] is false where the point is lost (a weak tensor at level 0,
// or a final position outside the image). n_setup[t] counts the window set-ups of target t (one per
// level, as a track of its own would form them) and n_iter[t] its iterations.
template <int RMAX, int NT>
__device__ void track_from(const uint8_t* fa, const uint8_t* pa, const uint8_t* const (&fb)[NT],
                           const uint8_t* const (&pb)[NT], int t0, int nt, const vs::LevelDesc& d, const LKConst& c,
                           float ux, float uy, float (&vx)[NT], float (&vy)[NT], bool (&ok)[NT],
                           uint32_t (&n_setup)[NT], uint32_t (&n_iter)[NT], float* red)
{
    const int lane = threadIdx.x & 63;
    const int gcol = lane % c.cols, grp = lane / c.cols;
    const bool active = grp < c.groups;
    const int qx = gcol - c.hw;
    const int qy0 = grp * c.rows - c.hw;                 // first window row of this lane
    int nrows = c.hw - qy0 + 1;                          // rows of this lane inside the window
    nrows = active ? (nrows < c.rows ? nrows : c.rows) : 0;
    nrows = nrows < 0 ? 0 : nrows;
    const int lane_off = grp * c.rows * 32 + gcol;       // the lane's first byte in a staged block
    uint32_t* stage = reinterpret_cast<uint32_t*>(red);

    ux = wave_uniform(ux);
    uy = wave_uniform(uy);
    float gx[NT], gy[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        gx[t] = gy[t] = 0.f;
        ok[t] = true;
    }
    for (int l = d.levels - 1; l >= 0; --l) {
        const Img A = level_img(fa, pa, d, l);
        const float sc = ldexpf(1.0f, -l);
        const float cx = ux * sc, cy = uy * sc;
        const float fx = floorf(cx), fy = floorf(cy);
        const float a = cx - fx, b = cy - fy;
        const int ix = (int)fx + qx, iy = (int)fy + qy0;

        // ---- window set-up: rows iy-1 .. iy+RMAX+1, columns ix-1 .. ix+2 of the previous frame, the
        // window's block starting at (fx - h - 1, fy - h - 1)
        const bool a_in = wave_all(!active || (ix - 1 >= 0 && ix + 2 <= A.w - 1 && iy - 1 >= 0 && iy + RMAX + 1 <= A.h - 1));
        const int bx = (int)fx - c.hw - 1, by = (int)fy - c.hw - 1;
        // the first target's first next-frame block is read with the set-up, so its residual sums
        // share the set-up's reduction: 3 tensor sums + 2 sums of I times the gradient + 8 residual sums
        const Img B0 = level_img(NT == 1 || t0 == 0 ? fb[0] : fb[NT - 1], NT == 1 || t0 == 0 ? pb[0] : pb[NT - 1], d, l);
        const float g0x = NT == 1 || t0 == 0 ? gx[0] : gx[NT - 1], g0y = NT == 1 || t0 == 0 ? gy[0] : gy[NT - 1];
        const int jx0 = (int)floorf(cx + g0x), jy0 = (int)floorf(cy + g0y);
        float I[RMAX], Ix[RMAX], Iy[RMAX];
        float qa[RMAX + 1], qb[RMAX + 1];
        bool both_staged = false;
        if constexpr (RMAX <= 7) {
            const int x0 = jx0 + qx, y0 = jy0 + qy0;
            both_staged = a_in && wave_all(!active || (x0 >= 0 && x0 + 1 <= B0.w - 1 && y0 >= 0 && y0 + RMAX <= B0.h - 1));
            if (both_staged) {
                if (c.full)
                    setup_staged<RMAX, false>(A, B0, bx, by, jx0 - c.hw, jy0 - c.hw, lane_off, a, b, nrows, active, red,
                                              I, Ix, Iy, qa, qb);
                else
                    setup_staged<RMAX, true>(A, B0, bx, by, jx0 - c.hw, jy0 - c.hw, lane_off, a, b, nrows, active, red,
                                             I, Ix, Iy, qa, qb);
            }
        }
        if (!both_staged) {
            if (c.full) {
                if (a_in)
                    window_samples<RMAX, true, false>(A, ix, iy, bx, by, lane_off, a, b, nrows, active, stage, I, Ix, Iy);
                else
                    window_samples<RMAX, false, false>(A, ix, iy, bx, by, lane_off, a, b, nrows, active, stage, I, Ix, Iy);
            } else {
                if (a_in)
                    window_samples<RMAX, true, true>(A, ix, iy, bx, by, lane_off, a, b, nrows, active, stage, I, Ix, Iy);
                else
                    window_samples<RMAX, false, true>(A, ix, iy, bx, by, lane_off, a, b, nrows, active, stage, I, Ix, Iy);
            }
            load_next_block<RMAX>(B0, jx0 + qx, jy0 + qy0, jx0 - c.hw, jy0 - c.hw, lane_off, active, stage, qa, qb);
        }
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
        float tot[13];
        wave_sums<16, 13>(v, tot, red);
        const float g11 = tot[0], g12 = tot[1], g22 = tot[2], Sx = tot[3], Sy = tot[4];
        float E[8];
        e_from_sums(Sx, tot[5], tot[6], tot[7], tot[8], E);
        e_from_sums(Sy, tot[9], tot[10], tot[11], tot[12], E + 4);
        const float tr = g11 + g22;
        // hardware square root (about 1 ulp): the value only enters the eigenvalue test
        const float sq = __builtin_amdgcn_sqrtf((g11 - g22) * (g11 - g22) + 4.0f * g12 * g12);
        const float lmax = 0.5f * (tr + sq);
        const float det = det2(g11, g22, g12);
        // lambda_min = det / lambda_max, so lambda_min / N >= min_eig is det >= (N min_eig) lambda_max
        // (no division). The tensor is 4 G and the residual sums 2 b (D = 2 grad I): the threshold
        // carries the factor 4, and G^-1 b = 2 (4 G)^-1 (2 b).
        const bool strong = uniform(lmax > 0.f ? det >= c.eig_thr * lmax : c.eig_thr <= 0.f);
#pragma unroll
        for (int ti = 0; ti < NT; ++ti) {
            // ti walks the slots t0 .. nt - 1 (one slot when NT == 1)
            const int t = NT == 1 ? 0 : t0 + ti;
            if (NT > 1 && t >= nt) break;
            ++n_setup[t];
            float nux = 0.f, nuy = 0.f;
            if (!strong) {
                if (l == 0) ok[t] = false;
            } else {
                // step = (4 G)^-1 (2 b) * 2 = H b with H = 2 adj(4 G) / det(4 G), formed once per level
                const float inv = 2.0f * __builtin_amdgcn_rcpf(det);
                const float h11 = g11 * inv, h12 = g12 * inv, h22 = g22 * inv;
                const Img B = (NT == 1 || t == 0) ? level_img(fb[0], pb[0], d, l)
                                                  : level_img(fb[NT - 1], pb[NT - 1], d, l);
                const float px0 = cx + gx[t], py0 = cy + gy[t];
                float cfx = floorf(px0), cfy = floorf(py0);   // the integer position of the current sums
                if (ti > 0) {
                    // a later target: its first block read like a reload, its sums added in the order of
                    // the set-up's reduction (16-lane chunks), as a track of its own adds them
                    const int jx = (int)cfx, jy = (int)cfy;
                    load_next_block<RMAX>(B, jx + qx, jy + qy0, jx - c.hw, jy - c.hw, lane_off, active, stage, qa, qb);
                    float e[16], t8[8];
                    residual_partials<RMAX>(Ix, Iy, qa, qb, e);
                    wave_sums<16, 8>(e, t8, red);
                    e_from_sums(Sx, t8[0], t8[1], t8[2], t8[3], E);
                    e_from_sums(Sy, t8[4], t8[5], t8[6], t8[7], E + 4);
                }
                for (int it = 0; it < c.max_iter; ++it) {
                    const float pxx = px0 + nux, pyy = py0 + nuy;
                    float ja = pxx - cfx, jb = pyy - cfy;
                    // the iterate left its pixel unless both fractions lie in [0, 1): as unsigned integers
                    // the bit patterns of [0, 1) are exactly those below 1.0's (negatives carry the sign bit)
                    if (uniform(__float_as_uint(ja) >= 0x3f800000u || __float_as_uint(jb) >= 0x3f800000u)) {
                        // the integer position moved: new block, new residual sums
                        const float jfx = floorf(pxx), jfy = floorf(pyy);
                        cfx = jfx;
                        cfy = jfy;
                        ja = pxx - jfx;
                        jb = pyy - jfy;
                        const int jx = (int)jfx, jy = (int)jfy;
                        load_next_block<RMAX>(B, jx + qx, jy + qy0, jx - c.hw, jy - c.hw, lane_off, active, stage, qa, qb);
                        float e[8], t8[8];
                        residual_partials<RMAX>(Ix, Iy, qa, qb, e);
                        wave_sums<8, 8>(e, t8, red);
                        e_from_sums(Sx, t8[0], t8[1], t8[2], t8[3], E);
                        e_from_sums(Sy, t8[4], t8[5], t8[6], t8[7], E + 4);
                    }
                    // b = E0 - ja E1 - jb E2 - ja jb E3 = (E0 - jb E2) - ja (E1 + jb E3)
                    const float b1 = fmaf(-ja, fmaf(jb, E[3], E[1]), fmaf(-jb, E[2], E[0]));
                    const float b2 = fmaf(-ja, fmaf(jb, E[7], E[5]), fmaf(-jb, E[6], E[4]));
                    const float ex = fmaf(h22, b1, -(h12 * b2));
                    const float ey = fmaf(h11, b2, -(h12 * b1));
                    nux += ex;
                    nuy += ey;
                    ++n_iter[t];
                    if (uniform(ex * ex + ey * ey < c.eps2)) break;
                }
            }
            // the guesses and results are the same in every lane: kept in scalar registers
            if (l > 0) {
                gx[t] = wave_uniform(2.0f * (gx[t] + nux));
                gy[t] = wave_uniform(2.0f * (gy[t] + nuy));
            } else {
                vx[t] = wave_uniform(ux + gx[t] + nux);
                vy[t] = wave_uniform(uy + gy[t] + nuy);
            }
        }
    }
#pragma unroll
    for (int t = 0; t < NT; ++t)
        if (!(vx[t] >= 0.f && vy[t] >= 0.f && vx[t] <= (float)(d.w[0] - 1) && vy[t] <= (float)(d.h[0] - 1))) ok[t] = false;
}

// one track of u from frame A into frame B
template <int RMAX>
__device__ __forceinline__ bool track_one(const uint8_t* fa, const uint8_t* pa, const uint8_t* fb, const uint8_t* pb,
                                          const vs::LevelDesc& d, const LKConst& c, float ux, float uy, float& vx,
                                          float& vy, uint32_t& n_setup, uint32_t& n_iter, float* red)
{
    const uint8_t* const fbs[1] = {fb};
    const uint8_t* const pbs[1] = {pb};
    float ox[1] = {vx}, oy[1] = {vy};
    bool ok[1];
    uint32_t ns[1] = {n_setup}, ni[1] = {n_iter};
    track_from<RMAX, 1>(fa, pa, fbs, pbs, 0, 1, d, c, ux, uy, ox, oy, ok, ns, ni, red);
    vx = ox[0];
    vy = oy[0];
    n_setup = ns[0];
    n_iter = ni[0];
    return ok[0];
}

// the round-trip error of the backward check, |b - u|, in one fixed operation order
__device__ __forceinline__ float fb_error(float bx, float by, float ux, float uy)
{
    const float dx = bx - ux, dy = by - uy;
    return sqrtf(fmaf(dx, dx, dy * dy));
}

// what one tracked item reads and writes; slot k's point is xy_prev[2k], its outputs at index k
struct LkItem {
    const uint8_t *fa, *pa, *fb, *pb;   // previous frame and pyramid, next frame and pyramid
    const float* xy_prev;
    const uint8_t* alive_prev;
    float* xy_next;
    uint8_t* status;
    float* fb_err;
    int32_t* n_valid;
    float* xy_chain;
    uint8_t* alive_chain;
};

// item i of a strided call: frames and pyramids at i * stride, records at g = i * istride
struct Strided {
    const uint8_t *prev_frames, *prev_pyrs, *next_frames, *next_pyrs;
    int64_t frame_stride, pyr_stride;
    int istride, capacity;
    const float* xy_prev;
    const uint8_t* alive_prev;
    float* xy_next;
    uint8_t* status;
    float* fb_err;
    int32_t* n_valid;
    float* xy_chain;
    uint8_t* alive_chain;
    __device__ __forceinline__ bool at(int i, LkItem& it) const
    {
        const int64_t g = (int64_t)i * istride, k = g * capacity;
        it.fa = prev_frames + i * frame_stride;
        it.pa = prev_pyrs + i * pyr_stride;
        it.fb = next_frames + i * frame_stride;
        it.pb = next_pyrs + i * pyr_stride;
        it.xy_prev = xy_prev + 2 * k;
        it.alive_prev = alive_prev ? alive_prev + k : nullptr;
        it.xy_next = xy_next + 2 * k;
        it.status = status + k;
        it.fb_err = fb_err ? fb_err + k : nullptr;
        it.n_valid = n_valid ? n_valid + g : nullptr;
        it.xy_chain = xy_chain ? xy_chain + 2 * k : nullptr;
        it.alive_chain = alive_chain ? alive_chain + k : nullptr;
        return true;
    }
};

// item i of a batched step: the pair (frame j - 1, frame j) of its stream, skipped at j = 0; the
// points tracked from frame j - 1 sit at [(j - 1) & 1] of the stream's point records, the tracked
// points are chained to [j & 1]
struct Step {
    vs::StepView v;
    __device__ __forceinline__ bool at(int i, LkItem& it) const
    {
        const vs::StepStream& d = v.s(i);
        const int64_t j = d.next_frame;
        if (j == 0) return false;
        const int cur = (int)(j & 1), prv = cur ^ 1;
        const int64_t cap = v.capacity;
        it.fa = v.frame(i, j - 1);
        it.pa = d.pyr + prv * v.pyr_bytes;
        it.fb = v.frame(i, j);
        it.pb = d.pyr + cur * v.pyr_bytes;
        it.xy_prev = d.pts + prv * cap * 2;
        it.alive_prev = d.alive + prv * cap;
        it.xy_next = d.dst;
        it.status = d.status;
        it.fb_err = d.fb_err;
        it.n_valid = d.n_valid;
        it.xy_chain = d.pts + cur * cap * 2;
        it.alive_chain = d.alive + cur * cap;
        return true;
    }
};

template <int RMAX, class A>
__device__ __forceinline__ void lk_body(const A& io, const vs::LevelDesc& d, int capacity, const LKConst& c, int fb,
                                        float fb_thresh, unsigned long long* work, int n_items, int by_xcd)
{
    // each wave of the workgroup tracks one point slot on its own (no barriers): slot = group *
    // waves + wave. All point slots of an item run on one XCD, so the overlapping windows of its
    // frame pair are shared in that XCD's L2.
    const int ppg = blockDim.x >> 6;
    const int groups = (capacity + ppg - 1) / ppg;
    int item, group;
    if (!vs::xcd_map(blockIdx.x, n_items, groups, by_xcd != 0, item, group)) return;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));   // wave-uniform
    const int slot = group * ppg + wave;
    if (slot >= capacity) return;
    LkItem it;
    if (!io.at(item, it)) return;
    const int lane = threadIdx.x & 63;
    extern __shared__ float lk_lds[];
    float* red = lk_lds + wave * WAVE_LDS_FLOATS;
    // the zero area read by lanes outside the window
    red[RED_FLOATS + lane] = 0.f;
    if (lane < ZERO_FLOATS - 64) red[RED_FLOATS + 64 + lane] = 0.f;
    wave_lds_sync();
    const int k = slot;
    const float ux = it.xy_prev[2 * k], uy = it.xy_prev[2 * k + 1];
    const bool alive = it.alive_prev ? it.alive_prev[k] != 0 : true;
    float vx = ux, vy = uy, err = __int_as_float(0x7fc00000);
    bool ok = false;
    uint32_t n_setup = 0, n_iter = 0;
    if (alive) {
        ok = track_one<RMAX>(it.fa, it.pa, it.fb, it.pb, d, c, ux, uy, vx, vy, n_setup, n_iter, red);
        if (ok && fb) {
            float bx = vx, by = vy;
            const bool okb = track_one<RMAX>(it.fb, it.pb, it.fa, it.pa, d, c, vx, vy, bx, by, n_setup, n_iter, red);
            err = fb_error(bx, by, ux, uy);
            ok = okb && err <= fb_thresh;
        }
    }
    if (lane == 0) {
        it.xy_next[2 * k] = vx;
        it.xy_next[2 * k + 1] = vy;
        it.status[k] = ok ? 1 : 0;
        if (it.fb_err) it.fb_err[k] = err;
        if (it.xy_chain) {
            it.xy_chain[2 * k] = vx;
            it.xy_chain[2 * k + 1] = vy;
        }
        if (it.alive_chain) it.alive_chain[k] = ok ? 1 : 0;
        if (ok && it.n_valid) atomicAdd(it.n_valid, 1);
        if (work && n_setup) {   // per-item counters: one address per item keeps the atomics uncontended
            atomicAdd(&work[2 * item], (unsigned long long)n_setup);
            atomicAdd(&work[2 * item + 1], (unsigned long long)n_iter);
        }
    }
}

// Windows of at most 7 rows per lane run five waves per SIMD (at most 96 VGPRs); larger windows keep
// the registers they need.
template <class A>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) void lk_kernel7(
    A io, vs::LevelDesc d, int capacity, LKConst c, int fb, float fb_thresh, unsigned long long* work, int n_items,
    int by_xcd)
{
    lk_body<7>(io, d, capacity, c, fb, fb_thresh, work, n_items, by_xcd);
}

template <class A>
__global__ __launch_bounds__(256) void lk_kernel16(A io, vs::LevelDesc d, int capacity, LKConst c, int fb,
                                                  float fb_thresh, unsigned long long* work, int n_items, int by_xcd)
{
    lk_body<16>(io, d, capacity, c, fb, fb_thresh, work, n_items, by_xcd);
}

// One call over chains of tracked pairs (vs_track_lk_segments). Item i holds the frames
// F(i, s) = frames + i * frame_stride + s * frame_step and the point records of its pair s at record
// i * istride + s. One wave carries one point slot of one item through the item's pairs: the forward
// track of the first pair, then for every later frame one window set-up that serves both the
// backward track of the pair ending there and the forward track of the pair starting there (a
// segment of 5 pairs forms 6 set-ups per point and level instead of 10). A pair skipped for too few
// valid points is only known once all of its points are done, so the call assumes none is; a gated
// call from the pair after a skipped one tracks the rest of that item again.
struct SegIO {
    const uint8_t *frames, *pyrs;
    int64_t frame_stride, pyr_stride, frame_step, pyr_step;
    int n, istride, capacity, first, pairs, last_pairs;
    float* xy;
    uint8_t* alive;
    float* dst;
    uint8_t* status;
    float* fb_err;
    int32_t* n_valid;
    const int32_t* gate;
    int gate_min;

    __device__ __forceinline__ int pairs_of(int i) const { return i == n - 1 ? last_pairs : pairs; }
    __device__ __forceinline__ bool gated_in(int i) const { return !gate || gate[(int64_t)i * istride] < gate_min; }
};

template <int RMAX>
__device__ __forceinline__ void lk_segment_body(const SegIO& io, const vs::LevelDesc& d, const LKConst& c, int fb,
                                                float fb_thresh, unsigned long long* work, int by_xcd)
{
    const int ppg = blockDim.x >> 6;
    const int groups = (io.capacity + ppg - 1) / ppg;
    int item, group;
    if (!vs::xcd_map(blockIdx.x, io.n, groups, by_xcd != 0, item, group)) return;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));   // wave-uniform
    const int slot = group * ppg + wave;
    if (slot >= io.capacity) return;
    const int last = io.pairs_of(item);
    if (io.first >= last || !io.gated_in(item)) return;
    const int lane = threadIdx.x & 63;
    extern __shared__ float lk_lds[];
    float* red = lk_lds + wave * WAVE_LDS_FLOATS;
    red[RED_FLOATS + lane] = 0.f;
    if (lane < ZERO_FLOATS - 64) red[RED_FLOATS + 64 + lane] = 0.f;
    wave_lds_sync();
    const uint8_t* f0 = io.frames + item * io.frame_stride;
    const uint8_t* p0 = io.pyrs + item * io.pyr_stride;
    const int64_t r0 = (int64_t)item * io.istride;
    const int cap = io.capacity;
    int s = io.first;
    // the point at the start of pair s, whether it entered the pair, and its forward track
    int64_t k = (r0 + s) * cap + slot;
    float px = io.xy[2 * k], py = io.xy[2 * k + 1];
    bool live = io.alive[k] != 0;
    float vx = px, vy = py;
    bool fok = false;
    uint32_t n_kept = 0, i_kept = 0, n_formed = 0;
    if (live) {
        uint32_t ns = 0, ni = 0;
        fok = track_one<RMAX>(f0 + s * io.frame_step, p0 + s * io.pyr_step, f0 + (s + 1) * io.frame_step,
                              p0 + (s + 1) * io.pyr_step, d, c, px, py, vx, vy, ns, ni, red);
        n_kept += ns;
        i_kept += ni;
        n_formed += ns;
    }
    for (; s < last; ++s) {
        k = (r0 + s) * cap + slot;
        const bool more = s + 1 < last;
        const uint8_t* fm = f0 + (s + 1) * io.frame_step;   // the frame pair s ends on
        const uint8_t* pm = p0 + (s + 1) * io.pyr_step;
        float nx = vx, ny = vy;                           // the next pair's forward track
        bool okn = false, ok_s = false;
        float err = __int_as_float(0x7fc00000);
        uint32_t ns[2] = {0u, 0u}, ni[2] = {0u, 0u};
        if (live && fok) {
            if (fb) {
                // backward into frame s and forward into frame s + 2 from the same windows of frame s + 1
                const uint8_t* const fts[2] = {f0 + s * io.frame_step, more ? fm + io.frame_step : fm};
                const uint8_t* const pts[2] = {p0 + s * io.pyr_step, more ? pm + io.pyr_step : pm};
                float ox[2] = {vx, vx}, oy[2] = {vy, vy};
                bool ok[2] = {false, false};
                track_from<RMAX, 2>(fm, pm, fts, pts, 0, more ? 2 : 1, d, c, vx, vy, ox, oy, ok, ns, ni, red);
                err = fb_error(ox[0], oy[0], px, py);
                ok_s = ok[0] && err <= fb_thresh;
                nx = ox[1];
                ny = oy[1];
                okn = ok[1];
            } else {
                ok_s = true;
                if (more)
                    okn = track_one<RMAX>(fm, pm, fm + io.frame_step, pm + io.pyr_step, d, c, vx, vy, nx, ny, ns[1],
                                          ni[1], red);
            }
        }
        n_kept += ns[0] + (ok_s ? ns[1] : 0u);
        i_kept += ni[0] + (ok_s ? ni[1] : 0u);
        n_formed += fb ? ns[0] : (ok_s ? ns[1] : 0u);
        if (lane == 0) {
            io.dst[2 * k] = vx;
            io.dst[2 * k + 1] = vy;
            io.status[k] = ok_s ? 1 : 0;
            if (io.fb_err) io.fb_err[k] = err;
            if (ok_s && io.n_valid) atomicAdd(io.n_valid + r0 + s, 1);
            if (more) {
                const int64_t kn = k + cap;
                io.xy[2 * kn] = vx;
                io.xy[2 * kn + 1] = vy;
                io.alive[kn] = ok_s ? 1 : 0;
            }
        }
        // pair s + 1 starts where pair s ended; a point lost in pair s stays there
        px = vx;
        py = vy;
        live = ok_s;
        if (ok_s) {
            vx = wave_uniform(nx);
            vy = wave_uniform(ny);
        }
        fok = ok_s && okn;
    }
    if (lane == 0 && work && n_formed) {
        atomicAdd(&work[3 * item], (unsigned long long)n_kept);
        atomicAdd(&work[3 * item + 1], (unsigned long long)i_kept);
        atomicAdd(&work[3 * item + 2], (unsigned long long)n_formed);
    }
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) void lk_segment_kernel7(
    SegIO io, vs::LevelDesc d, LKConst c, int fb, float fb_thresh, unsigned long long* work, int by_xcd)
{
    lk_segment_body<7>(io, d, c, fb, fb_thresh, work, by_xcd);
}

__global__ __launch_bounds__(256) void lk_segment_kernel16(SegIO io, vs::LevelDesc d, LKConst c, int fb,
                                                          float fb_thresh, unsigned long long* work, int by_xcd)
{
    lk_segment_body<16>(io, d, c, fb, fb_thresh, work, by_xcd);
}

// points (waves) per workgroup of a gated segment call: the most the kernels' 256-thread bound allows
constexpr int LK_MAX_THREADS = 256;
constexpr int GATED_POINTS_PER_GROUP = LK_MAX_THREADS / 64;

// clears the valid counts of the pairs a segment call makes (items the gate lets in) and its counters
__global__ void zero_segment_counters(SegIO io, unsigned long long* work)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= io.n) return;
    if (io.n_valid && io.gated_in(i)) {
        const int last = io.pairs_of(i);
        for (int s = io.first; s < last; ++s) io.n_valid[(int64_t)i * io.istride + s] = 0;
    }
    if (work) {
        work[3 * i] = 0;
        work[3 * i + 1] = 0;
        work[3 * i + 2] = 0;
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

LKConst lk_const(const vs_lk_params& p)
{
    LKConst c;
    c.hw = p.win_half;
    c.cols = 2 * c.hw + 1;
    c.groups = 64 / c.cols;
    c.rows = (c.cols + c.groups - 1) / c.groups;
    c.nwin = c.cols * c.cols;
    c.max_iter = p.max_iter;
    c.eps2 = p.eps * p.eps;
    c.full = c.groups * c.rows == c.cols && c.rows == (c.rows <= 7 ? 7 : 16);
    c.eig_thr = (float)(4.0 * (double)p.min_eig * (double)c.nwin);
    return c;
}

template <class A>
int launch_lk(const A& io, const vs_pyramid& layout, int capacity, const LKConst& c, const vs_lk_params& p,
              unsigned long long* wk, int n, hipStream_t s)
{
    const vs::LevelDesc d = vs::level_desc(layout);
    const bool by_xcd = n >= vs::xcd_min_items(vs::XCD_LK);
    const int ppg = vs::lk_points_per_group();
    const int64_t nblk = vs::xcd_grid(n, (capacity + ppg - 1) / ppg, by_xcd);
    if (nblk > 0x7fffffff) return vs::set_error(VS_ERR_INVALID, "vs_track_lk: grid too large");
    const unsigned grid = (unsigned)nblk;
    const unsigned threads = 64u * (unsigned)ppg;
    const size_t lds = sizeof(float) * WAVE_LDS_FLOATS * (size_t)ppg;
    if (c.rows <= 7)
        lk_kernel7<A><<<grid, threads, lds, s>>>(io, d, capacity, c, p.fb, p.fb_thresh, wk, n, by_xcd);
    else
        lk_kernel16<A><<<grid, threads, lds, s>>>(io, d, capacity, c, p.fb, p.fb_thresh, wk, n, by_xcd);
    return vs::check_launch("vs_track_lk");
}

// checks shared by the tracking entry points
int check_lk(const vs_pyramid& layout, const vs_lk_params& p, int capacity, int n)
{
    if (layout.levels < 1 || layout.levels > VS_MAX_LEVELS)
        return vs::set_error(VS_ERR_UNSUPPORTED, "vs_track_lk: levels out of range");
    if (capacity > VS_MAX_CORNERS) return vs::set_error(VS_ERR_UNSUPPORTED, "vs_track_lk: capacity > %d", VS_MAX_CORNERS);
    if (p.win_half < 1 || p.win_half > 15) return vs::set_error(VS_ERR_UNSUPPORTED, "vs_track_lk: win_half must be 1..15");
    if (p.max_iter < 1 || !(p.eps >= 0.f) || !(p.min_eig >= 0.f) || !(p.fb_thresh >= 0.f))
        return vs::set_error(VS_ERR_INVALID, "vs_track_lk: bad parameters");
    if (n > 65535) return vs::set_error(VS_ERR_INVALID, "vs_track_lk: more than 65535 items");
    if ((int64_t)layout.pitch[0] * layout.height[0] >= ((int64_t)1 << 31) || layout.pitch[0] >= (1 << 24))
        return vs::set_error(VS_ERR_UNSUPPORTED, "vs_track_lk: frame larger than 2 GiB or rows of 16 MiB");
    return VS_OK;
}

}  // namespace

namespace vs {

// the tracking of every item of a batched step with j > 0 (its n_valid is cleared by the step's
// set-up kernel)
int step_track(const StepView& v, int n, const vs_pyramid& L, const vs_lk_params& p, hipStream_t s)
{
    if (n <= 0) return VS_OK;
    const int e = check_lk(L, p, v.capacity, n);
    if (e) return e;
    return launch_lk(Step{v}, L, v.capacity, lk_const(p), p, nullptr, n, s);
}

}  // namespace vs

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
    const int ec = check_lk(*layout, *p, capacity, n);
    if (ec) return ec;
    const LKConst c = lk_const(*p);
    hipStream_t s = vs::as_stream(stream);
    unsigned long long* wk = reinterpret_cast<unsigned long long*>(work);
    if (n_valid || wk) {
        zero_counters<<<(n + 255) / 256, 256, 0, s>>>(n_valid, n, istride, wk);
        int e = vs::check_launch("vs_track_lk(zero)");
        if (e) return e;
    }
    const Strided io{prev_frames, prev_pyrs, next_frames, next_pyrs, frame_stride, pyr_stride, istride, capacity,
                     xy_prev, alive_prev, xy_next, status, fb_err, n_valid, xy_chain, alive_chain};
    return launch_lk(io, *layout, capacity, c, *p, wk, n, s);
}

extern "C" int vs_track_lk_segments(const uint8_t* frames, const uint8_t* pyrs, int64_t frame_stride,
                                    int64_t pyr_stride, int64_t frame_step, int64_t pyr_step, int32_t n,
                                    int32_t istride, int32_t pairs, int32_t last_pairs, int32_t first,
                                    const vs_pyramid* layout, int32_t capacity, const vs_lk_params* p, float* xy,
                                    uint8_t* alive, float* dst, uint8_t* status, float* fb_err, int32_t* n_valid,
                                    const int32_t* gate, int32_t gate_min, uint64_t* work, void* stream)
{
    if (!layout || !p) return vs::set_error(VS_ERR_INVALID, "vs_track_lk_segments: null argument");
    if (n < 0 || capacity < 0 || istride < 1 || pairs < 0 || last_pairs < 0 || last_pairs > pairs || first < 0 ||
        pairs > istride)
        return vs::set_error(VS_ERR_INVALID, "vs_track_lk_segments: bad count, stride or pair range");
    if (n == 0 || capacity == 0 || first >= pairs) return VS_OK;
    if (!frames || (layout->levels > 1 && !pyrs) || !xy || !alive || !dst || !status)
        return vs::set_error(VS_ERR_INVALID, "vs_track_lk_segments: null argument");
    const int ec = check_lk(*layout, *p, capacity, n);
    if (ec) return ec;
    const LKConst c = lk_const(*p);
    hipStream_t s = vs::as_stream(stream);
    unsigned long long* wk = reinterpret_cast<unsigned long long*>(work);
    const SegIO io{frames, pyrs, frame_stride, pyr_stride, frame_step, pyr_step, n, istride, capacity, first, pairs,
                   last_pairs, xy, alive, dst, status, fb_err, n_valid, gate, gate_min};
    if (n_valid || wk) {
        zero_segment_counters<<<(n + 255) / 256, 256, 0, s>>>(io, wk);
        const int e = vs::check_launch("vs_track_lk_segments(zero)");
        if (e) return e;
    }
    const vs::LevelDesc d = vs::level_desc(*layout);
    const bool by_xcd = n >= vs::xcd_min_items(vs::XCD_LK);
    // a gated call usually lets few items in: larger workgroups make the ones gated out cheap to dispatch
    const int ppg = gate ? GATED_POINTS_PER_GROUP : vs::lk_points_per_group();
    const int64_t nblk = vs::xcd_grid(n, (capacity + ppg - 1) / ppg, by_xcd);
    if (nblk > 0x7fffffff) return vs::set_error(VS_ERR_INVALID, "vs_track_lk_segments: grid too large");
    const unsigned threads = 64u * (unsigned)ppg;
    if (threads > (unsigned)LK_MAX_THREADS) return vs::set_error(VS_ERR_INVALID, "vs_track_lk_segments: workgroup too large");
    const size_t lds = sizeof(float) * WAVE_LDS_FLOATS * (size_t)ppg;
    if (c.rows <= 7)
        lk_segment_kernel7<<<(unsigned)nblk, threads, lds, s>>>(io, d, c, p->fb, p->fb_thresh, wk, by_xcd);
    else
        lk_segment_kernel16<<<(unsigned)nblk, threads, lds, s>>>(io, d, c, p->fb, p->fb_thresh, wk, by_xcd);
    return vs::check_launch("vs_track_lk_segments");
}
