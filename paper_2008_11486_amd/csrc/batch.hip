// Many stacks of uneven frame counts and sizes in one launch per phase.
//
// The host turns the stacks into one table of work items, grouped by phase:
//
//   CAL        calibrate a band of rows of one frame into the workspace
//   MEANPART   sum MEAN_ROWS template rows of the calibrated reference
//   MEANFINAL  template mean of the reference
//   SCORE      one tile of partial correlation scores (the stack's tuned launch shape)
//   SSCORE     the same for windows of side <= 5 (one tile of 240 x 256 template pixels per item)
//   SUM        64 candidate scores of one frame from its tile partials
//   PICK       argmax, runner-up, parabola of one frame
//   RECT       common overlap of the stack from its offsets
//   SHIFT      a 16-row strip of one frame's bilinear shift onto the overlap
//   COMB*      sigma-clipped mean of a block of pixel columns (one launch per frame-count
//              class: up to 16, 32, 48, 64 or 128 frames)
//   FUSE*      for a block of output pixels of a stack of up to 48 frames without a
//              bad-pixel map: every frame's aligned values (bilinear taps of the
//              calibrated frames, in registers) and the clipped mean, in one pass (one
//              launch per frame-count class; such stacks take no SHIFT or COMB item and
//              keep no aligned frames)
//
// Each phase is one kernel launch with one workgroup per item over all stacks; the
// stream orders the phases, so every dependency is met at a kernel boundary and no
// workgroup waits for another.  The search items go out in an XCD-aware order.  Each
// item calls the same device routines as the stage-wise kernels with the same launch
// shape, so results are bit-identical to them.  Items of the shift and combine phases
// are counted for the whole frame (the overlap is only known on the device) and those
// outside the overlap return at once.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "calibrate_core.h"
#include "combine_core.h"
#include "common.h"
#include "register_core.h"
#include "register_plan.h"
#include "shift_core.h"

namespace rd {

ScoreArgs make_score_args(const RegPlan &p, const float *ref, const float *frames, const int32_t *centers,
                          const double *mean, double *partial, int32_t W, int32_t H, int32_t N, int32_t R,
                          int32_t Rmax, int32_t tx0, int32_t ty0, int32_t tw, int32_t th, int32_t skip);

constexpr int BATCH_THREADS = 512;
constexpr int COMB_PX16 = 4;    // pixel columns per thread of the up-to-16-frame combine
constexpr int COMB_PX32 = 2;    // ... of the up-to-32-frame combine

// Plane stride (floats) of the aligned-frame workspace for an overlap of w x h: padded
// to 4 floats so that every frame's plane starts 16-byte aligned.
__host__ __device__ inline int64_t al_plane(int64_t w, int64_t h) { return (w * h + 3) & ~(int64_t)3; }

enum ItemType : int32_t {
    IT_CAL = 0, IT_MEANPART, IT_MEANFINAL, IT_SCORE, IT_SSCORE, IT_SUM, IT_PICK, IT_RECT, IT_SHIFT, IT_MASK,
    IT_COMB16, IT_COMB32, IT_COMB48, IT_COMBDEEP, IT_COMB16M, IT_COMB32M, IT_COMB48M, IT_COMBMISS,
    IT_FUSE16, IT_FUSE32, IT_FUSE48
};
constexpr int N_PHASES = IT_FUSE48 + 1;

struct Item {
    int32_t type, stack, a, pad;
};

struct StackDev {
    // caller buffers
    const uint16_t *raw;
    int64_t rrp, rfp;
    const float *dark, *flat;
    int64_t crp;
    const float *bias;     // or NULL
    const uint8_t *mask;   // bad-pixel map [H][W] or NULL
    float *out;
    int32_t *out_rect;
    reduce_offset_t *offsets;
    int64_t *n_rej;
    // sizes and parameters
    int32_t W, H, N, ref, R, max_iters, integer_mode, cal_vec, K;
    float ksigma;
    // workspace
    float *cal;           // [N][H][W]
    float *al;            // [N][h][w] aligned frames (room for [N][H][W])
    double *mean_parts;   // [n_mean_parts]
    double *mean;         // [1]
    double *partial;      // [N-1][n_tiles][D*D]
    double *scores;       // [N-1][D*D]
    float *soffs;         // [N][2] offsets applied by the shift
    int32_t *rect;        // [4]
    int32_t n_mean_parts;
    ScoreArgs sa;
};

struct BatchArgs {
    const Item *items;
    const StackDev *stacks;
};

// ---- phase kernels: one workgroup per item ------------------------------------------------
__global__ __launch_bounds__(CAL_BLOCK) void batch_cal(BatchArgs a, int32_t first)
{
    const Item it = a.items[first + blockIdx.x];
    const StackDev &s = a.stacks[it.stack];
    const int64_t i = (int64_t)it.a * CAL_BLOCK + threadIdx.x;
    if (s.cal_vec)
        calibrate_group8(s.raw, s.rrp, s.rfp, s.bias, s.dark, s.flat, s.crp, s.cal, s.W, s.H, s.N, i);
    else
        calibrate_pixel(s.raw, s.rrp, s.rfp, s.bias, s.dark, s.flat, s.crp, s.cal, s.W, s.H, s.N, i);
}

__global__ __launch_bounds__(MEAN_THREADS) void batch_meanpart(BatchArgs a, int32_t first)
{
    __shared__ double scratch[MEAN_THREADS / 64];
    const Item it = a.items[first + blockIdx.x];
    const StackDev &s = a.stacks[it.stack];
    const double v = tmpl_part_sum(s.sa.ref, s.W, s.sa.tx0, s.sa.ty0, s.sa.tw, s.sa.th, it.a, scratch);
    if (threadIdx.x == 0) s.mean_parts[it.a] = v;
}

__global__ __launch_bounds__(MEAN_THREADS) void batch_meanfinal(BatchArgs a, int32_t first)
{
    __shared__ double scratch[MEAN_THREADS / 64];
    const Item it = a.items[first + blockIdx.x];
    const StackDev &s = a.stacks[it.stack];
    const double m =
        tmpl_mean_of_parts(s.mean_parts, s.n_mean_parts, (double)s.sa.tw * (double)s.sa.th, scratch);
    if (threadIdx.x == 0) *s.mean = m;
}

// One launch per group of stacks that share a search shape (register block K, threads,
// LDS), with exactly that workgroup size and LDS, as the stage-wise launch uses.
template <int K>
__global__ __launch_bounds__(BATCH_THREADS) void batch_score(BatchArgs a, int32_t first, int32_t count)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const Item it = a.items[first + xcd_logical_id((int32_t)blockIdx.x, count)];
    const StackDev &s = a.stacks[it.stack];
    score_tile<K>(s.sa, it.a, smem);
}

__global__ __launch_bounds__(SMALL_COLS) void batch_score_small(BatchArgs a, int32_t first)
{
    __shared__ __align__(16) float fl[SMALL_LDS_FLOATS];
    const Item it = a.items[first + blockIdx.x];
    const StackDev &s = a.stacks[it.stack];
    small_dispatch(s.sa.D, [&](auto Dc) { score_small_tile<decltype(Dc)::value>(s.sa, it.a, fl); });
}

__global__ __launch_bounds__(64 * SUM_WAVES) void batch_sum(BatchArgs a, int32_t first)
{
    __shared__ double part[SUM_WAVES][64];
    const Item it = a.items[first + blockIdx.x];
    const StackDev &s = a.stacks[it.stack];
    const int32_t D = s.sa.D;
    const int32_t blocks = (D * D + 63) / 64;
    const int32_t k = it.a / blocks, cb = it.a - k * blocks;
    sum_candidate_block(s.partial + (int64_t)k * s.sa.n_tiles * D * D, s.sa.n_tiles, D, s.R, s.R, 0, 0, cb,
                        s.scores + (int64_t)k * D * D, part);
}

__global__ __launch_bounds__(256) void batch_pick(BatchArgs a, int32_t first)
{
    __shared__ Best scratch[4];
    const Item it = a.items[first + blockIdx.x];
    const StackDev &s = a.stacks[it.stack];
    const int32_t D = s.sa.D, k = it.a;
    const int32_t kf = k + (k >= s.ref ? 1 : 0);
    pick_frame(s.scores + (int64_t)k * D * D, D, s.R, s.R, 0, 0, s.offsets + kf, scratch);
}

__global__ void batch_rect(BatchArgs a, int32_t first)
{
    if (threadIdx.x != 0) return;
    const StackDev &s = a.stacks[a.items[first + blockIdx.x].stack];
    // reference frame: offset 0 by definition
    reduce_offset_t z;
    z.dx = z.dy = 0;
    z.sx = z.sy = 0.0f;
    z.peak = 0.0;
    z.second = -INFINITY;
    z.margin = INFINITY;
    z.flags = 0;
    z.pad = 0;
    s.offsets[s.ref] = z;
    double xl = -1e300, xh = 1e300, yl = -1e300, yh = 1e300;
    for (int32_t k = 0; k < s.N; ++k) {
        float sx = 0.0f, sy = 0.0f;
        if (k != s.ref) {
            const reduce_offset_t o = s.offsets[k];
            sx = s.integer_mode ? (float)o.dx : o.sx;
            sy = s.integer_mode ? (float)o.dy : o.sy;
        }
        s.soffs[2 * k] = sx;
        s.soffs[2 * k + 1] = sy;
        const double lo_x = ceil(-(double)sx), hi_x = floor((double)(s.W - 1) - (double)sx);
        const double lo_y = ceil(-(double)sy), hi_y = floor((double)(s.H - 1) - (double)sy);
        xl = lo_x > xl ? lo_x : xl;
        xh = hi_x < xh ? hi_x : xh;
        yl = lo_y > yl ? lo_y : yl;
        yh = hi_y < yh ? hi_y : yh;
    }
    int32_t r[4] = {0, 0, 0, 0};  // no overlap: empty output
    if (xl <= xh && yl <= yh) {
        r[0] = (int32_t)xl;
        r[1] = (int32_t)yl;
        r[2] = (int32_t)(xh - xl) + 1;
        r[3] = (int32_t)(yh - yl) + 1;
    }
    for (int i = 0; i < 4; ++i) {
        s.rect[i] = r[i];
        s.out_rect[i] = r[i];
    }
}

__global__ __launch_bounds__(SH_BLOCK) void batch_shift(BatchArgs a, int32_t first)
{
    const Item it = a.items[first + blockIdx.x];
    const StackDev &s = a.stacks[it.stack];
    const int32_t x0 = s.rect[0], y0 = s.rect[1], w = s.rect[2], h = s.rect[3];
    const int32_t xblks = (int32_t)ceil_div(s.W, (int64_t)SH_BLOCK * SH_VEC);
    const int32_t strips = (int32_t)ceil_div(s.H, SH_ROWS);
    const int32_t k = it.a / (strips * xblks);
    const int32_t r = it.a - k * strips * xblks;
    const int32_t strip = r / xblks, xblk = r - strip * xblks;
    if (w < 1 || h < 1) return;
    const int vs = shift_vec_store(w, reinterpret_cast<uintptr_t>(s.al));
    const bool aligned = s.W % 4 == 0;
    const int64_t pstride = al_plane(w, h);
    if (s.integer_mode)
        shift_strip<true, SH_VEC>(s.cal, s.al, s.W, s.H, k, s.soffs[2 * k], s.soffs[2 * k + 1], strip, xblk, x0, y0,
                                  w, h, pstride, vs, aligned);
    else
        shift_strip<false, SH_VEC>(s.cal, s.al, s.W, s.H, k, s.soffs[2 * k], s.soffs[2 * k + 1], strip, xblk, x0,
                                   y0, w, h, pstride, vs, aligned);
}

// Sigma-clipped mean of block it.a of the stack's overlap; PX pixel columns per thread
// when the overlap plane allows vector loads, else one.
template <int MAXV, int PX, bool MISS>
__global__ __launch_bounds__(COMB_TILE) void batch_comb(BatchArgs a, int32_t first)
{
    const Item it = a.items[first + blockIdx.x];
    const StackDev &s = a.stacks[it.stack];
    const int64_t plane = (int64_t)s.rect[2] * s.rect[3];
    const int64_t pstride = al_plane(s.rect[2], s.rect[3]);
    // the aligned planes are padded to 4 floats; the output image needs PX-float alignment
    const bool vec = PX > 1 && (reinterpret_cast<uintptr_t>(s.out) & (uintptr_t)(4 * PX - 1)) == 0;
    const int64_t blocks = vec ? ceil_div(plane, (int64_t)COMB_TILE * PX) : ceil_div(plane, (int64_t)COMB_TILE);
    if (it.a >= blocks) return;  // uniform over the workgroup
    unsigned dropped;
    if (vec)
        dropped = combine_cols_block<MAXV, PX, MISS>(s.al, plane, pstride, s.N, (double)s.ksigma, s.max_iters,
                                                     s.out, nullptr, it.a);
    else
        dropped = combine_cols_block<MAXV, 1, MISS>(s.al, plane, pstride, s.N, (double)s.ksigma, s.max_iters, s.out,
                                                    nullptr, it.a);
    if (s.n_rej) {
        const unsigned total = block_sum_u32(dropped);
        if (threadIdx.x == 0 && total) atomicAdd(reinterpret_cast<unsigned long long *>(s.n_rej),
                                                 (unsigned long long)total);
    }
}

// ---- shift + clipped mean in one pass ---------------------------------------------------
// Q + 1 taps of one frame row at columns c0 .. c0 + Q (clamped into the row), as shift_strip
// reads them: two 16-byte loads from the aligned column c0 - (c0 & 3) when they lie inside
// the row (rows 16-byte aligned), else one float at a time.
template <int Q>
__device__ __forceinline__ void row_taps(const float *__restrict__ row, int32_t c0, int32_t W, bool aligned,
                                         float (&t)[Q + 1])
{
    static_assert(Q <= 4, "two 16-byte loads cover the taps");
    const int32_t al = c0 & 3, b = c0 - al;
    if (aligned && b >= 0 && b + 8 <= W) {
        const float4 u = *reinterpret_cast<const float4 *>(row + b);
        const float4 v = *reinterpret_cast<const float4 *>(row + b + 4);
        const float raw[8] = {u.x, u.y, u.z, u.w, v.x, v.y, v.z, v.w};
        switch (al) {
        case 0:
#pragma unroll
            for (int e = 0; e <= Q; ++e) t[e] = raw[e];
            break;
        case 1:
#pragma unroll
            for (int e = 0; e <= Q; ++e) t[e] = raw[1 + e];
            break;
        case 2:
#pragma unroll
            for (int e = 0; e <= Q; ++e) t[e] = raw[2 + e];
            break;
        default:
#pragma unroll
            for (int e = 0; e <= Q; ++e) t[e] = raw[3 + e];
            break;
        }
    } else {
#pragma unroll
        for (int e = 0; e <= Q; ++e) t[e] = row[clampi(c0 + e, 0, W - 1)];
    }
}

// Aligned values of frame k at the Q output pixels (u0 + e, v) of one row of the overlap,
// exactly as shift_strip makes them: taps in rows clamp(y0 + v + iy) and the one below
// (when the vertical fraction is not zero), columns clamp(x0 + u + ix) and the one to the
// right (when the horizontal fraction is not zero), from the calibrated frame.
template <int Q>
__device__ __forceinline__ void aligned_row(const StackDev &s, int32_t k, int32_t u0, int32_t v, int32_t x0,
                                            int32_t y0, bool aligned, float (&r)[Q])
{
    const ShiftSetup ss = shift_setup(s.soffs[2 * k], s.soffs[2 * k + 1]);
    const bool integer = s.integer_mode != 0;
    const bool step = ss.a > 0.0;
    const bool down = !integer && ss.b > 0.0;
    const int32_t j = clampi(y0 + v + ss.iy, 0, s.H - 1);
    const int32_t j1 = clampi(down ? j + 1 : j, 0, s.H - 1);
    const int32_t c0 = x0 + u0 + ss.ix;
    const float *f = s.cal + (int64_t)k * s.W * s.H;
    float t0[Q + 1], t1[Q + 1];
    row_taps<Q>(f + (int64_t)j * s.W, c0, s.W, aligned, t0);
    if (j1 != j)
        row_taps<Q>(f + (int64_t)j1 * s.W, c0, s.W, aligned, t1);
    else
#pragma unroll
        for (int e = 0; e <= Q; ++e) t1[e] = t0[e];
#pragma unroll
    for (int e = 0; e < Q; ++e) {
        if (integer) {
            r[e] = t0[e];
        } else {
            const float f10 = step ? t0[e + 1] : t0[e];
            const float f11 = step ? t1[e + 1] : t1[e];
            r[e] = bilerp(ss.a, ss.b, t0[e], f10, t1[e], f11);
        }
    }
}

// A block of FUSE_PX consecutive output pixels (linear index over the overlap) of every
// frame: first the aligned values, FUSE_Q pixels of one frame per work unit, all units of
// the block spread over the workgroup (many loads in flight) into an LDS tile
// [N][FUSE_PX]; then one thread per pixel clips its column of the tile in registers (the
// queue of combine_cols_block made this phase slower: 22.2 -> 24.0 ms per step on the
// 64-stack workload, so every column is clipped in place).
constexpr int FUSE_PX = 256;
constexpr int FUSE_Q = 4;
static_assert(FUSE_PX == COMB_TILE, "one pixel per thread in the clip");

template <int MAXV>
__global__ __launch_bounds__(COMB_TILE) void batch_fused(BatchArgs a, int32_t first)
{
    extern __shared__ float tile[];  // [N][FUSE_PX]
    const Item it = a.items[first + blockIdx.x];
    const StackDev &s = a.stacks[it.stack];
    const int32_t x0 = s.rect[0], y0 = s.rect[1], w = s.rect[2], h = s.rect[3];
    const int64_t plane = (int64_t)w * h;
    const int64_t pb = (int64_t)it.a * FUSE_PX;
    if (pb >= plane) return;  // uniform over the workgroup
    const bool aligned = s.W % 4 == 0;  // calibrated rows start 16-byte aligned
    const int t = threadIdx.x;
    constexpr int UNITS = FUSE_PX / FUSE_Q;         // work units per frame
    constexpr int KSTEP = COMB_TILE / UNITS;        // frames taken together
    // thread t: pixels q * FUSE_Q .. + FUSE_Q - 1 of the block, frames k0, k0 + KSTEP, ...
    const int q = t % UNITS, k0 = t / UNITS;
    const int64_t p0 = pb + q * FUSE_Q;
    const int32_t v0 = (int32_t)(p0 / w), u0 = (int32_t)(p0 - (int64_t)v0 * w);
    const bool one_row = p0 + FUSE_Q <= plane && u0 + FUSE_Q <= w;
#pragma unroll 4
    for (int32_t k = k0; k < s.N; k += KSTEP) {
        float r[FUSE_Q] = {0.0f, 0.0f, 0.0f, 0.0f};
        if (one_row) {
            aligned_row<FUSE_Q>(s, k, u0, v0, x0, y0, aligned, r);
        } else {
#pragma unroll
            for (int c = 0; c < FUSE_Q; ++c) {
                const int64_t p = p0 + c;
                if (p < plane) {
                    const int32_t v = (int32_t)(p / w);
                    float r1[1];
                    aligned_row<1>(s, k, (int32_t)(p - (int64_t)v * w), v, x0, y0, aligned, r1);
                    r[c] = r1[0];
                }
            }
        }
        *reinterpret_cast<float4 *>(tile + (int64_t)k * FUSE_PX + q * FUSE_Q) = make_float4(r[0], r[1], r[2], r[3]);
    }
    __syncthreads();
    float x[MAXV];
#pragma unroll
    for (int i = 0; i < MAXV; ++i) x[i] = i < s.N ? tile[i * FUSE_PX + t] : 0.0f;
    KeptBits<MAXV> kept;
    unsigned dropped = 0;
    const float res = clip_registers<MAXV>(x, s.N, (double)s.ksigma, s.max_iters, kept, dropped);
    const int64_t p = pb + t;
    if (p < plane) s.out[p] = res;
    else dropped = 0;
    if (s.n_rej) {
        const unsigned total = block_sum_u32(dropped);
        if (threadIdx.x == 0 && total)
            atomicAdd(reinterpret_cast<unsigned long long *>(s.n_rej), (unsigned long long)total);
    }
}

// Row v = it.a / N of frame k = it.a % N of a stack with a bad-pixel map (the frames
// of a row consecutive, so that they share the map rows in L2): aligned values that
// read a bad pixel become NaN (missing in the combine).
__global__ __launch_bounds__(256) void batch_mask(BatchArgs a, int32_t first, int32_t count)
{
    // XCD-aware order: the frames of a row, and neighbouring rows, on one XCD (one L2)
    const Item it = a.items[first + xcd_logical_id((int32_t)blockIdx.x, count)];
    const StackDev &s = a.stacks[it.stack];
    const int32_t v = it.a / s.N, k = it.a - v * s.N;
    const int32_t x0 = s.rect[0], y0 = s.rect[1], w = s.rect[2], h = s.rect[3];
    if (v >= h) return;  // uniform over the workgroup
    const ShiftSetup ss = shift_setup(s.soffs[2 * k], s.soffs[2 * k + 1]);
    float *row = s.al + (int64_t)k * al_plane(w, h) + (int64_t)v * w;
    for (int32_t u = threadIdx.x; u < w; u += blockDim.x)
        if (reads_bad_pixel(s.mask, s.W, s.H, ss, s.integer_mode != 0, x0 + u, y0 + v)) row[u] = __builtin_nanf("");
}

// Stacks of 49 - 128 frames (MISS: stacks with a bad-pixel map, any depth): block it.a
// of 64 pixel columns, values in LDS [N][64] (the launch sizes the tile for the deepest
// stack of the phase).
template <bool MISS>
__global__ __launch_bounds__(COMB_DEEP_PX) __attribute__((amdgpu_waves_per_eu(3))) void batch_comb_deep(BatchArgs a, int32_t first)
{
    extern __shared__ float tile[];
    const Item it = a.items[first + blockIdx.x];
    const StackDev &s = a.stacks[it.stack];
    const int64_t plane = (int64_t)s.rect[2] * s.rect[3];
    if (it.a >= ceil_div(plane, (int64_t)COMB_DEEP_PX)) return;  // uniform over the workgroup
    unsigned dropped = combine_deep_block<MISS>(s.al, plane, al_plane(s.rect[2], s.rect[3]), s.N, (double)s.ksigma,
                                                s.max_iters, s.out, nullptr, it.a, tile);
    if (s.n_rej) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) dropped += __shfl_xor(dropped, off, 64);
        if (threadIdx.x == 0 && dropped)
            atomicAdd(reinterpret_cast<unsigned long long *>(s.n_rej), (unsigned long long)dropped);
    }
}

__global__ void batch_reset(int64_t *const *n_rej, int32_t n_stacks)
{
    for (int32_t i = threadIdx.x; i < n_stacks; i += blockDim.x)
        if (n_rej[i]) *n_rej[i] = 0;
}

// ---- host side ---------------------------------------------------------------------------
static size_t al(size_t b) { return (b + 255) & ~(size_t)255; }

struct StackLayout {
    RegPlan plan;
    size_t cal, al, mean_parts, mean, partial, scores, soffs, rect;
    int32_t count[N_PHASES];
};

struct ScoreGroup {
    int32_t K, threads;
    size_t lds;
    std::vector<int32_t> stacks;  // by decreasing search work
    int32_t first, count;         // item range within the SCORE phase
};

struct BatchLayout {
    std::vector<StackLayout> st;
    size_t items, stacks, nrej_ptrs, total;
    int32_t n_items;
    int32_t first[N_PHASES], count[N_PHASES];
    size_t score_lds;
    size_t spec_ws = 0, spec = 0;  // workspace of the largest spectral search and its offset
    int32_t deep_n = 0;  // deepest stack of the deep combine phase
    int32_t miss_n = 0;  // deepest stack of the combine with missing values
    std::vector<ScoreGroup> groups;
};

static double search_cost(const StackLayout &sl)
{
    const RegPlan &p = sl.plan;
    return (double)sl.count[IT_SCORE] * p.BR * p.TX * p.C;
}

static int validate(const reduce_stack_t *stacks, int32_t n)
{
    for (int32_t i = 0; i < n; ++i) {
        const reduce_stack_t &s = stacks[i];
        const std::string who = "reduce_stack_batch: stack " + std::to_string(i);
        if (!s.raw || !s.dark || !s.flat || !s.out || !s.out_rect || !s.offsets)
            return fail(REDUCE_ERR_NULL, who + ": NULL buffer");
        if (s.W < 1 || s.H < 1 || s.N < 1) return fail(REDUCE_ERR_SHAPE, who + ": W, H, N must be >= 1");
        if (s.raw_row_pitch < s.W || s.raw_frame_pitch < s.raw_row_pitch * (int64_t)(s.H - 1) + s.W ||
            s.cal_row_pitch < s.W)
            return fail(REDUCE_ERR_SHAPE, who + ": pitch smaller than the frame");
        if (s.N > COMB_MAX_N_COLS) return fail(REDUCE_ERR_UNSUPPORTED, who + ": N above 128");
        if (s.ref_index < 0 || s.ref_index >= s.N) return fail(REDUCE_ERR_RANGE, who + ": ref_index out of range");
        if (s.radius < 0 || s.W - 2 * s.radius < 1 || s.H - 2 * s.radius < 1)
            return fail(REDUCE_ERR_RANGE, who + ": radius leaves no template");
        if (!(s.ksigma > 0.0f) || s.max_iters < 0) return fail(REDUCE_ERR_RANGE, who + ": bad clip parameters");
        if (reg_plan(s.W, s.H, s.radius, s.radius).D == 0)
            return fail(REDUCE_ERR_UNSUPPORTED, who + ": radius too large for any launch shape");
        if (s.search != REDUCE_SEARCH_DIRECT && s.search != REDUCE_SEARCH_SPECTRAL)
            return fail(REDUCE_ERR_RANGE, who + ": unknown search");
        if (s.search == REDUCE_SEARCH_SPECTRAL && s.N > 1 &&
            (s.radius < 1 || reduce_register_fft_ws(s.W, s.H, s.N, s.radius) == 0))
            return fail(REDUCE_ERR_UNSUPPORTED, who + ": no search through row spectra for these sizes");
    }
    return REDUCE_OK;
}

// The stack registers through row spectra (a stack of one frame has nothing to register).
static bool spectral(const reduce_stack_t &s) { return s.search == REDUCE_SEARCH_SPECTRAL && s.N > 1; }

// Dark subtraction takes 8-pixel groups when rows, pitches and pointers allow it.
static bool cal_vec_ok(const reduce_stack_t &s)
{
    const auto a16 = [](const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; };
    return s.W % CAL_VEC == 0 && s.raw_row_pitch % CAL_VEC == 0 && s.raw_frame_pitch % CAL_VEC == 0 &&
           s.cal_row_pitch % 4 == 0 && a16(s.raw) && a16(s.dark) && a16(s.flat) && (!s.bias || a16(s.bias));
}

static BatchLayout layout_of(const reduce_stack_t *stacks, int32_t n)
{
    BatchLayout L;
    size_t off = 0;
    L.score_lds = 0;
    for (int p = 0; p < N_PHASES; ++p) L.count[p] = 0;
    for (int32_t i = 0; i < n; ++i) {
        const reduce_stack_t &s = stacks[i];
        StackLayout sl{};  // every phase count starts at zero
        sl.plan = reg_plan(s.W, s.H, s.radius, s.radius);
        const RegPlan &p = sl.plan;
        const int64_t fp = (int64_t)s.W * s.H;
        const int32_t nreg = s.N - 1;
        // a stack of up to 48 frames without a bad-pixel map takes the fused phase (no
        // aligned frames in the workspace)
        const bool fuse = s.mask == nullptr && s.N <= 48;
        sl.cal = off;
        off += al(sizeof(float) * fp * s.N);
        sl.al = off;
        if (!fuse) off += al(sizeof(float) * al_plane(s.W, s.H) * s.N);
        const int32_t n_mean_parts = (int32_t)ceil_div(s.H - 2 * s.radius, MEAN_ROWS);
        sl.mean_parts = off;
        off += al(sizeof(double) * n_mean_parts);
        sl.mean = off;
        off += 256;
        const bool spec = spectral(s);
        const int32_t ndir = spec ? 0 : nreg;  // frames of the direct search
        sl.partial = off;
        off += al(sizeof(double) * (size_t)std::max(ndir, 0) * p.n_tiles * p.D * p.D);
        sl.scores = off;
        off += al(sizeof(double) * (size_t)std::max(ndir, 0) * p.D * p.D);
        if (spec) L.spec_ws = std::max(L.spec_ws, reduce_register_fft_ws(s.W, s.H, s.N, s.radius));
        sl.soffs = off;
        off += al(sizeof(float) * 2 * s.N);
        sl.rect = off;
        off += 256;
        sl.count[IT_CAL] = (int32_t)ceil_div(cal_vec_ok(s) ? fp / CAL_VEC : fp, CAL_BLOCK);
        sl.count[IT_MEANPART] = n_mean_parts;
        sl.count[IT_MEANFINAL] = 1;
        sl.count[IT_SCORE] = p.K != 0 ? ndir * p.wg_per_frame : 0;
        sl.count[IT_SSCORE] = p.K == 0 ? ndir * p.wg_per_frame : 0;
        sl.count[IT_SUM] = ndir * (int32_t)ceil_div((int64_t)p.D * p.D, 64);
        sl.count[IT_PICK] = ndir;
        sl.count[IT_RECT] = 1;
        sl.count[IT_SHIFT] =
            fuse ? 0 : s.N * (int32_t)ceil_div(s.H, SH_ROWS) * (int32_t)ceil_div(s.W, (int64_t)SH_BLOCK * SH_VEC);
        // enough clip items for the whole frame (the overlap is only known on the device),
        // PX columns per thread when the output image allows PX-float stores
        const int px = s.N <= 16 ? COMB_PX16 : s.N <= 32 ? COMB_PX32 : 1;
        const bool vec = px > 1 && (reinterpret_cast<uintptr_t>(s.out) & (uintptr_t)(4 * px - 1)) == 0;
        const int32_t comb_blocks = (int32_t)ceil_div(fp, (int64_t)COMB_TILE * (vec ? px : 1));
        // a stack with a bad-pixel map has its aligned values masked and takes the combine
        // that leaves missing values out
        const bool miss = s.mask != nullptr;
        sl.count[IT_MASK] = miss ? s.N * s.H : 0;
        const int32_t c16 = s.N <= 16 ? comb_blocks : 0;
        const int32_t c32 = s.N > 16 && s.N <= 32 ? comb_blocks : 0;
        const int32_t c48 = s.N > 32 && s.N <= 48 ? comb_blocks : 0;
        if (fuse) {
            const int32_t fb = (int32_t)ceil_div(fp, (int64_t)FUSE_PX);
            sl.count[IT_FUSE16] = s.N <= 16 ? fb : 0;
            sl.count[IT_FUSE32] = s.N > 16 && s.N <= 32 ? fb : 0;
            sl.count[IT_FUSE48] = s.N > 32 ? fb : 0;
        }
        const int32_t deep_blocks = s.N > 48 ? (int32_t)ceil_div(fp, (int64_t)COMB_DEEP_PX) : 0;
        sl.count[miss ? IT_COMB16M : IT_COMB16] = fuse ? 0 : c16;
        sl.count[miss ? IT_COMB32M : IT_COMB32] = fuse ? 0 : c32;
        sl.count[miss ? IT_COMB48M : IT_COMB48] = fuse ? 0 : c48;
        sl.count[miss ? IT_COMBMISS : IT_COMBDEEP] = deep_blocks;
        if (s.N > 48) (miss ? L.miss_n : L.deep_n) = std::max(miss ? L.miss_n : L.deep_n, s.N);
        for (int q = 0; q < N_PHASES; ++q) L.count[q] += sl.count[q];
        if (ndir > 0 && p.K != 0) L.score_lds = std::max(L.score_lds, p.lds);
        L.st.push_back(sl);
    }
    int64_t total = 0;
    for (int q = 0; q < N_PHASES; ++q) {
        L.first[q] = (int32_t)total;
        total += L.count[q];
    }
    L.n_items = total > INT32_MAX ? -1 : (int32_t)total;
    // search groups by shape, in order of first appearance; stacks within a group by cost
    int32_t next = L.first[IT_SCORE];
    for (int32_t i = 0; i < n; ++i) {
        const StackLayout &sl = L.st[i];
        if (sl.count[IT_SCORE] == 0) continue;
        ScoreGroup *g = nullptr;
        for (ScoreGroup &c : L.groups)
            if (c.K == sl.plan.K && c.threads == sl.plan.threads && c.lds == sl.plan.lds) g = &c;
        if (!g) {
            L.groups.push_back(ScoreGroup{sl.plan.K, sl.plan.threads, sl.plan.lds, {}, 0, 0});
            g = &L.groups.back();
        }
        g->stacks.push_back(i);
    }
    for (ScoreGroup &g : L.groups) {
        std::stable_sort(g.stacks.begin(), g.stacks.end(),
                         [&](int32_t x, int32_t y) { return search_cost(L.st[x]) > search_cost(L.st[y]); });
        g.first = next;
        g.count = 0;
        for (int32_t i : g.stacks) g.count += L.st[i].count[IT_SCORE];
        next += g.count;
    }
    L.spec = off;  // one spectral search at a time
    off += al(L.spec_ws);
    L.items = off;
    off += al(sizeof(Item) * (size_t)std::max<int64_t>(total, 0));
    L.stacks = off;
    off += al(sizeof(StackDev) * (size_t)n);
    L.nrej_ptrs = off;
    off += al(sizeof(int64_t *) * (size_t)n);
    L.total = off;
    return L;
}

struct BatchEntry {
    uint64_t hash = 0;
    bool ready = false;
    std::vector<unsigned char> host;  // uploaded descriptor bytes (kept alive with the entry)
};

static std::mutex g_batch_mu;
static std::map<void *, BatchEntry> g_entries;  // by workspace address

static uint64_t fnv1a(const void *p, size_t n, uint64_t h = 1469598103934665603ull)
{
    const unsigned char *b = static_cast<const unsigned char *>(p);
    for (size_t i = 0; i < n; ++i) {
        h ^= b[i];
        h *= 1099511628211ull;
    }
    return h;
}

// Host image of the descriptors of every stack and of the item table.
static int build_descriptors(const reduce_stack_t *stacks, int32_t n, void *ws, const BatchLayout &L,
                             BatchEntry *e)
{
    unsigned char *base = static_cast<unsigned char *>(ws);
    std::vector<StackDev> sd(n);
    std::vector<int64_t *> nrej(n);
    for (int32_t i = 0; i < n; ++i) {
        const reduce_stack_t &st = stacks[i];
        const StackLayout &sl = L.st[i];
        StackDev &d = sd[i];
        d.raw = st.raw;
        d.rrp = st.raw_row_pitch;
        d.rfp = st.raw_frame_pitch;
        d.dark = st.dark;
        d.flat = st.flat;
        d.bias = st.bias;
        d.mask = st.mask;
        d.crp = st.cal_row_pitch;
        d.out = st.out;
        d.out_rect = st.out_rect;
        d.offsets = st.offsets;
        d.n_rej = st.n_rej;
        nrej[i] = st.n_rej;
        d.W = st.W;
        d.H = st.H;
        d.N = st.N;
        d.ref = st.ref_index;
        d.R = st.radius;
        d.max_iters = st.max_iters;
        d.integer_mode = st.integer_mode ? 1 : 0;
        d.cal_vec = cal_vec_ok(st) ? 1 : 0;
        d.K = sl.plan.K;
        d.ksigma = st.ksigma;
        d.cal = reinterpret_cast<float *>(base + sl.cal);
        d.al = reinterpret_cast<float *>(base + sl.al);
        d.mean_parts = reinterpret_cast<double *>(base + sl.mean_parts);
        d.mean = reinterpret_cast<double *>(base + sl.mean);
        d.partial = reinterpret_cast<double *>(base + sl.partial);
        d.scores = reinterpret_cast<double *>(base + sl.scores);
        d.soffs = reinterpret_cast<float *>(base + sl.soffs);
        d.rect = reinterpret_cast<int32_t *>(base + sl.rect);
        d.n_mean_parts = sl.count[IT_MEANPART];
        const int32_t R = st.radius;
        const float *ref = d.cal + (int64_t)d.ref * st.W * st.H;
        d.sa = make_score_args(sl.plan, ref, d.cal, nullptr, d.mean, d.partial, st.W, st.H, std::max(st.N - 1, 1), R,
                               R, R, R, st.W - 2 * R, st.H - 2 * R, d.ref);
    }
    // the table, phase by phase; within a phase the largest stacks first
    std::vector<int32_t> order(n);
    for (int32_t i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
        const auto cost = [&](int32_t z) {
            const RegPlan &p = L.st[z].plan;
            return (double)(L.st[z].count[IT_SCORE] + L.st[z].count[IT_SSCORE]) * p.BR * p.TX * p.C +
                   (double)L.st[z].count[IT_SHIFT] + (double)L.st[z].count[IT_FUSE16] +
                   (double)L.st[z].count[IT_FUSE32] + (double)L.st[z].count[IT_FUSE48];
        };
        return cost(x) > cost(y);
    });
    std::vector<Item> items;
    items.reserve(L.n_items);
    for (int q = 0; q < N_PHASES; ++q) {
        if (q == IT_SCORE) {
            for (const ScoreGroup &g : L.groups)
                for (int32_t i : g.stacks)
                    for (int32_t a = 0; a < L.st[i].count[q]; ++a) items.push_back({q, i, a, 0});
            continue;
        }
        for (int32_t i : order)
            for (int32_t a = 0; a < L.st[i].count[q]; ++a) items.push_back({q, i, a, 0});
    }
    if ((int32_t)items.size() != L.n_items) return fail(REDUCE_ERR_SHAPE, "reduce_stack_batch: item count");
    e->host.assign(L.total - L.items, 0);
    std::memcpy(e->host.data(), items.data(), sizeof(Item) * items.size());
    std::memcpy(e->host.data() + (L.stacks - L.items), sd.data(), sizeof(StackDev) * sd.size());
    std::memcpy(e->host.data() + (L.nrej_ptrs - L.items), nrej.data(), sizeof(int64_t *) * nrej.size());
    return REDUCE_OK;
}

template <typename F>
static void score_dispatch_host(int K, F &&f)
{
    switch (K) {
    case 5: f(std::integral_constant<int, 5>{}); break;
    case 9: f(std::integral_constant<int, 9>{}); break;
    case 12: f(std::integral_constant<int, 12>{}); break;
    case 17: f(std::integral_constant<int, 17>{}); break;
    case 18: f(std::integral_constant<int, 18>{}); break;
    default: f(std::integral_constant<int, 22>{}); break;
    }
}

static int launch_phases(const reduce_stack_t *stacks, int32_t n, void *ws, const BatchLayout &L, hipStream_t s)
{
    unsigned char *base = static_cast<unsigned char *>(ws);
    BatchArgs a;
    a.items = reinterpret_cast<const Item *>(base + L.items);
    a.stacks = reinterpret_cast<const StackDev *>(base + L.stacks);
    int64_t *const *nrej_dev = reinterpret_cast<int64_t *const *>(base + L.nrej_ptrs);
    hipLaunchKernelGGL(batch_reset, dim3(1), dim3(256), 0, s, nrej_dev, n);
    if (L.count[IT_CAL] > 0)
        hipLaunchKernelGGL(batch_cal, dim3(L.count[IT_CAL]), dim3(CAL_BLOCK), 0, s, a, L.first[IT_CAL]);
    if (L.count[IT_MEANPART] > 0)
        hipLaunchKernelGGL(batch_meanpart, dim3(L.count[IT_MEANPART]), dim3(MEAN_THREADS), 0, s, a,
                           L.first[IT_MEANPART]);
    hipLaunchKernelGGL(batch_meanfinal, dim3(L.count[IT_MEANFINAL]), dim3(MEAN_THREADS), 0, s, a,
                       L.first[IT_MEANFINAL]);
    if (L.count[IT_SCORE] > 0) {
        for (const ScoreGroup &g : L.groups) {
            ProfScope prof("batch_score", s);  // one record per dispatch
            score_dispatch_host(g.K, [&](auto Kc) {
                constexpr int K = decltype(Kc)::value;
                hipLaunchKernelGGL(batch_score<K>, dim3(g.count), dim3(g.threads), g.lds, s, a, g.first, g.count);
            });
        }
    }
    if (L.count[IT_SSCORE] > 0)
        hipLaunchKernelGGL(batch_score_small, dim3(L.count[IT_SSCORE]), dim3(SMALL_COLS), 0, s, a,
                           L.first[IT_SSCORE]);
    if (L.count[IT_SUM] > 0)
        hipLaunchKernelGGL(batch_sum, dim3(L.count[IT_SUM]), dim3(64 * SUM_WAVES), 0, s, a, L.first[IT_SUM]);
    if (L.count[IT_PICK] > 0)
        hipLaunchKernelGGL(batch_pick, dim3(L.count[IT_PICK]), dim3(256), 0, s, a, L.first[IT_PICK]);
    // the stacks that register through row spectra, one after the other in the shared space
    for (int32_t i = 0; i < n; ++i) {
        const reduce_stack_t &st = stacks[i];
        if (!spectral(st)) continue;
        ProfScope prof("batch_spectral", s);
        const float *cal = reinterpret_cast<const float *>(base + L.st[i].cal);
        const int rc = reduce_register_fft(cal + (int64_t)st.ref_index * st.W * st.H, cal, st.W, st.H, st.N,
                                           st.radius, st.offsets, nullptr, nullptr, base + L.spec, L.spec_ws, s);
        if (rc != REDUCE_OK) return rc;
    }
    hipLaunchKernelGGL(batch_rect, dim3(L.count[IT_RECT]), dim3(64), 0, s, a, L.first[IT_RECT]);
    {
        ProfScope prof("batch_shift", s);
        if (L.count[IT_SHIFT] > 0)
            hipLaunchKernelGGL(batch_shift, dim3(L.count[IT_SHIFT]), dim3(SH_BLOCK), 0, s, a, L.first[IT_SHIFT]);
    }
    if (L.count[IT_MASK] > 0)
        hipLaunchKernelGGL(batch_mask, dim3(L.count[IT_MASK]), dim3(256), 0, s, a, L.first[IT_MASK],
                           L.count[IT_MASK]);
    {
        ProfScope prof("batch_comb", s);
        if (L.count[IT_COMB16] > 0)
            hipLaunchKernelGGL((batch_comb<16, COMB_PX16, false>), dim3(L.count[IT_COMB16]), dim3(COMB_TILE), 0, s,
                               a, L.first[IT_COMB16]);
        if (L.count[IT_COMB32] > 0)
            hipLaunchKernelGGL((batch_comb<32, COMB_PX32, false>), dim3(L.count[IT_COMB32]), dim3(COMB_TILE), 0, s,
                               a, L.first[IT_COMB32]);
        if (L.count[IT_COMB48] > 0)
            hipLaunchKernelGGL((batch_comb<48, 1, false>), dim3(L.count[IT_COMB48]), dim3(COMB_TILE), 0, s, a,
                               L.first[IT_COMB48]);
        if (L.count[IT_COMB16M] > 0)
            hipLaunchKernelGGL((batch_comb<16, COMB_PX16, true>), dim3(L.count[IT_COMB16M]), dim3(COMB_TILE), 0, s,
                               a, L.first[IT_COMB16M]);
        if (L.count[IT_COMB32M] > 0)
            hipLaunchKernelGGL((batch_comb<32, COMB_PX32, true>), dim3(L.count[IT_COMB32M]), dim3(COMB_TILE), 0, s,
                               a, L.first[IT_COMB32M]);
        if (L.count[IT_COMB48M] > 0)
            hipLaunchKernelGGL((batch_comb<48, 1, true>), dim3(L.count[IT_COMB48M]), dim3(COMB_TILE), 0, s, a,
                               L.first[IT_COMB48M]);
        if (L.count[IT_COMBDEEP] > 0)
            hipLaunchKernelGGL(batch_comb_deep<false>, dim3(L.count[IT_COMBDEEP]), dim3(COMB_DEEP_PX),
                               sizeof(float) * (L.deep_n - COMB_DEEP_REG) * COMB_DEEP_PX, s, a, L.first[IT_COMBDEEP]);
        if (L.count[IT_COMBMISS] > 0)
            hipLaunchKernelGGL(batch_comb_deep<true>, dim3(L.count[IT_COMBMISS]), dim3(COMB_DEEP_PX),
                               sizeof(float) * (L.miss_n - COMB_DEEP_REG) * COMB_DEEP_PX, s, a, L.first[IT_COMBMISS]);
    }
    if (L.count[IT_FUSE16] + L.count[IT_FUSE32] + L.count[IT_FUSE48] > 0) {
        ProfScope prof("batch_fused", s);
        // the tile holds the frames of the class's deepest stack
        if (L.count[IT_FUSE16] > 0)
            hipLaunchKernelGGL(batch_fused<16>, dim3(L.count[IT_FUSE16]), dim3(COMB_TILE),
                               sizeof(float) * FUSE_PX * 16, s, a, L.first[IT_FUSE16]);
        if (L.count[IT_FUSE32] > 0)
            hipLaunchKernelGGL(batch_fused<32>, dim3(L.count[IT_FUSE32]), dim3(COMB_TILE),
                               sizeof(float) * FUSE_PX * 32, s, a, L.first[IT_FUSE32]);
        if (L.count[IT_FUSE48] > 0)
            hipLaunchKernelGGL(batch_fused<48>, dim3(L.count[IT_FUSE48]), dim3(COMB_TILE),
                               sizeof(float) * FUSE_PX * 48, s, a, L.first[IT_FUSE48]);
    }
    return check_launch("reduce_stack_batch");
}

}  // namespace rd

using namespace rd;

extern "C" size_t reduce_stack_batch_ws(const reduce_stack_t *stacks, int32_t n)
{
    if (!stacks || n < 1) return 0;
    if (validate(stacks, n) != REDUCE_OK) return 0;
    return layout_of(stacks, n).total;
}

extern "C" int reduce_stack_batch(const reduce_stack_t *stacks, int32_t n, void *ws, size_t ws_bytes, void *stream)
{
    if (!stacks) return fail(REDUCE_ERR_NULL, "reduce_stack_batch: NULL stacks");
    if (n < 1) return fail(REDUCE_ERR_SHAPE, "reduce_stack_batch: no stacks");
    const int v = validate(stacks, n);
    if (v != REDUCE_OK) return v;
    const BatchLayout L = layout_of(stacks, n);
    if (L.n_items < 0) return fail(REDUCE_ERR_UNSUPPORTED, "reduce_stack_batch: too many work items");
    for (int q = 0; q < N_PHASES; ++q)
        if (L.count[q] > 0x7fffffff / 2) return fail(REDUCE_ERR_UNSUPPORTED, "reduce_stack_batch: too many items");
    if (L.score_lds > 65536) return fail(REDUCE_ERR_UNSUPPORTED, "reduce_stack_batch: search tile above 64 KB");
    if (!ws || ws_bytes < L.total)
        return fail(REDUCE_ERR_WORKSPACE, "reduce_stack_batch: workspace needs " + std::to_string(L.total) + " bytes");
    hipStream_t s = as_stream(stream);

    // the host image of the descriptors is rebuilt only when the stacks or their launch
    // shapes change; it is uploaded into the workspace on every call
    uint64_t h = fnv1a(stacks, sizeof(reduce_stack_t) * (size_t)n);
    for (const StackLayout &sl : L.st) h = fnv1a(&sl.plan, sizeof(RegPlan), h);
    h = fnv1a(&L.total, sizeof(L.total), h);
    std::lock_guard<std::mutex> lk(g_batch_mu);
    BatchEntry &e = g_entries[ws];
    if (!e.ready || e.hash != h) {
        // an earlier call on this workspace may still read the old descriptors
        if (e.ready && hipStreamSynchronize(s) != hipSuccess)
            return fail(REDUCE_ERR_HIP, "reduce_stack_batch: synchronize before new descriptors");
        e = BatchEntry{};
        const int rc = build_descriptors(stacks, n, ws, L, &e);
        if (rc != REDUCE_OK) {
            g_entries.erase(ws);
            return rc;
        }
        e.hash = h;
        e.ready = true;
    }
    if (hipMemcpyAsync(static_cast<unsigned char *>(ws) + L.items, e.host.data(), e.host.size(),
                       hipMemcpyHostToDevice, s) != hipSuccess)
        return fail(REDUCE_ERR_HIP, "reduce_stack_batch: descriptor upload");
    ProfScope prof("stack_batch", s);
    return launch_phases(stacks, n, ws, L, s);
}
