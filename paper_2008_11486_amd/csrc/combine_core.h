// Device routine of the sigma-clipped mean over one pixel column held by a group of
// L lanes; used by the stage-wise combine kernel and by the fused batch kernel so
// both evaluate identical operations in identical order.
#pragma once

#include <type_traits>

#include "common.h"

namespace rd {

constexpr int COMB_TILE = 256;
constexpr int COMB_MAX_N = 48;        // LDS tile [N][256] floats stays within 48 KB
constexpr int COMB_MAX_N_COLS = 128;  // one lane per column: the column in registers

template <int MAXV>
struct ClipResult {
    float mean;      // mean of the kept values, rounded to float
    uint64_t kept;   // bit i: value lane + L*i is kept
    int dropped;     // values dropped over all iterations (whole group)
};

template <int L>
__device__ __forceinline__ double group_sum(double v)
{
#pragma unroll
    for (int off = 1; off < L; off <<= 1) v += __shfl_xor(v, off, L);
    return v;
}

template <int L>
__device__ __forceinline__ int group_sum(int v)
{
#pragma unroll
    for (int off = 1; off < L; off <<= 1) v += __shfl_xor(v, off, L);
    return v;
}

// Iterative clip: mean m and population sigma of the kept values, drop |x - m| >
// ksigma * sigma (all decided against the same m, sigma), stop when nothing drops
// or after max_iters passes, return the mean of what is kept.  Lane `lane` of the
// group owns the values col[(lane + L*i) * COMB_TILE], read from LDS on every pass
// (the compiler barrier keeps them from being hoisted into registers).  With L = 1
// the sums run over the frames in index order.
template <int L, int MAXV>
__device__ __forceinline__ ClipResult<MAXV> clip_column(const float *col, int32_t N, int lane, double ksigma,
                                                        int32_t max_iters)
{
    uint64_t kept = 0;
#pragma unroll
    for (int i = 0; i < MAXV; ++i)
        if (lane + L * i < N) kept |= (1ull << i);
    int n = N;
    int dropped = 0;
    for (int32_t it = 0; it < max_iters; ++it) {
        asm volatile("" ::: "memory");
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < MAXV; ++i)
            if ((kept >> i) & 1ull) s = __dadd_rn(s, (double)col[(lane + L * i) * COMB_TILE]);
        s = group_sum<L>(s);
        const double m = s / (double)n;
        double q = 0.0;
#pragma unroll
        for (int i = 0; i < MAXV; ++i)
            if ((kept >> i) & 1ull) {
                const double d = __dsub_rn((double)col[(lane + L * i) * COMB_TILE], m);
                q = __dadd_rn(q, __dmul_rn(d, d));
            }
        q = group_sum<L>(q);
        const double thr = __dmul_rn(ksigma, sqrt(q / (double)n));
        int drop = 0;
#pragma unroll
        for (int i = 0; i < MAXV; ++i)
            if (((kept >> i) & 1ull) && fabs(__dsub_rn((double)col[(lane + L * i) * COMB_TILE], m)) > thr) {
                kept &= ~(1ull << i);
                ++drop;
            }
        drop = group_sum<L>(drop);
        n -= drop;
        dropped += drop;
        if (drop == 0) break;
    }
    asm volatile("" ::: "memory");
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < MAXV; ++i)
        if ((kept >> i) & 1ull) s = __dadd_rn(s, (double)col[(lane + L * i) * COMB_TILE]);
    s = group_sum<L>(s);
    ClipResult<MAXV> r;
    r.mean = (float)(s / (double)n);
    r.kept = kept;
    r.dropped = dropped;
    return r;
}

// Clip the COMB_TILE pixel columns staged in LDS (tile[k * COMB_TILE + px] = value of
// frame k at pixel p0 + px) with groups of L lanes; the first COMB_TILE threads take
// part.  Writes out[p0 + px] and the keep mask; returns the values this thread
// dropped (counted in each group's lane 0).
template <int L, int MAXV>
__device__ __forceinline__ unsigned clip_tile(const float *tile, int64_t p0, int64_t plane, int32_t N,
                                              double ksigma, int32_t max_iters, float *out, uint8_t *keep)
{
    const int t = threadIdx.x;
    if (t >= COMB_TILE) return 0u;
    const int lane = t % L;
    const int group = t / L;
    constexpr int GROUPS = COMB_TILE / L;
    unsigned dropped_here = 0;
    for (int r = 0; r < L; ++r) {
        const int px = group + GROUPS * r;
        const int64_t p = p0 + px;
        ClipResult<MAXV> res = clip_column<L, MAXV>(tile + px, N, lane, ksigma, max_iters);
        if (p < plane) {
            if (lane == 0) out[p] = res.mean;
            if (keep) {
#pragma unroll
                for (int i = 0; i < MAXV; ++i) {
                    const int k = lane + L * i;
                    if (k < N) keep[k * plane + p] = (uint8_t)((res.kept >> i) & 1u);
                }
            }
            if (lane == 0) dropped_here += (unsigned)res.dropped;
        }
    }
    return dropped_here;
}

// Dispatch on the lanes per column; MAXV covers N <= COMB_MAX_N.
template <typename F>
__device__ __forceinline__ void lanes_dispatch(int L, int32_t N, F &&f)
{
    switch (L) {
    case 1:
        if (N <= 16) f(std::integral_constant<int, 1>{}, std::integral_constant<int, 16>{});
        else if (N <= 32) f(std::integral_constant<int, 1>{}, std::integral_constant<int, 32>{});
        else f(std::integral_constant<int, 1>{}, std::integral_constant<int, 48>{});
        break;
    case 2: f(std::integral_constant<int, 2>{}, std::integral_constant<int, 24>{}); break;
    case 4: f(std::integral_constant<int, 4>{}, std::integral_constant<int, 12>{}); break;
    case 8: f(std::integral_constant<int, 8>{}, std::integral_constant<int, 6>{}); break;
    case 16: f(std::integral_constant<int, 16>{}, std::integral_constant<int, 3>{}); break;
    case 32: f(std::integral_constant<int, 32>{}, std::integral_constant<int, 2>{}); break;
    default: f(std::integral_constant<int, 64>{}, std::integral_constant<int, 1>{}); break;
    }
}

// Sum of one unsigned per thread over a 256-thread workgroup.
__device__ __forceinline__ unsigned block_sum_u32(unsigned v)
{
    __shared__ unsigned part[COMB_TILE / 64];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    unsigned t = 0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += part[i];
    return t;
}

// Kept flags of up to MAXV values, one bit each (i is a compile-time index after
// unrolling, so the word and the bit are fixed).
template <int MAXV>
struct KeptBits {
    static constexpr int W = (MAXV + 63) / 64;
    uint64_t w[W];
    __device__ __forceinline__ bool get(int i) const { return ((w[i >> 6] >> (i & 63)) & 1ull) != 0; }
    __device__ __forceinline__ void clear(int i) { w[i >> 6] &= ~(1ull << (i & 63)); }
    __device__ __forceinline__ void first(int32_t N)  // values 0 .. N-1 kept
    {
#pragma unroll
        for (int j = 0; j < W; ++j) {
            const int32_t r = N - 64 * j;
            w[j] = r >= 64 ? ~0ull : r <= 0 ? 0ull : ((1ull << r) - 1ull);
        }
    }
};


// One thread per pixel column, the column's values read through x(i) (registers, or
// the thread's own slice of LDS).  The arithmetic is that of clip_column with one
// lane: sums in frame order in double, m = s / n, q = sum of (x - m)^2, threshold
// ksigma * sqrt(q / n), drop |x - m| > threshold.  Two shortcuts leave every result
// unchanged: the largest |x - m| of the q pass decides whether the drop pass is
// needed at all, and when an iteration drops nothing its own mean is the final mean.
// With FENCE a compiler barrier at each pass keeps values read from LDS from being
// held in registers across passes.
template <bool FENCE>
__device__ __forceinline__ void clip_fence()
{
    if (FENCE) asm volatile("" ::: "memory");
}

// With ALL (every value kept: the first iteration without missing values) the passes
// carry no per-value selects: the values past N are zero (the loads fill them so), which
// adds exactly nothing to a sum that starts at +0 (such a sum is never -0), and their
// deviations are multiplied by the uniform weight 0 (1 for i < N, an exact product) so
// they add exactly nothing to q and cannot raise the largest deviation.
template <int MAXV, bool ALL, bool FENCE, typename X>
__device__ __forceinline__ void clip_pass(X x, const KeptBits<MAXV> &kept, int32_t N, int n, double &s, double &m,
                                          double &q, double &dmax)
{
    clip_fence<FENCE>();
    s = 0.0;
#pragma unroll
    for (int i = 0; i < MAXV; ++i)
        if (ALL || kept.get(i)) s = __dadd_rn(s, (double)x(i));
    m = s / (double)n;
    q = 0.0;
    dmax = 0.0;
    clip_fence<FENCE>();
#pragma unroll
    for (int i = 0; i < MAXV; ++i)
        if (ALL || kept.get(i)) {
            double d = __dsub_rn((double)x(i), m);
            if (ALL) d = __dmul_rn(d, (double)min(max(N - i, 0), 1));
            q = __dadd_rn(q, __dmul_rn(d, d));
            dmax = fmax(dmax, fabs(d));
        }
}

// Clip one column; returns the mean and updates kept / dropped.
// With MISS, NaN values are missing: never kept, not counted as dropped, and n counts
// the others (a pixel with none gives NaN).
template <int MAXV, bool FENCE, bool MISS, typename X>
__device__ __forceinline__ float clip_values(X x, int32_t N, double ksigma, int32_t max_iters, KeptBits<MAXV> &kept,
                                             unsigned &dropped)
{
    kept.first(N);
    int n = N;
    if (MISS) {
#pragma unroll
        for (int i = 0; i < MAXV; ++i)
            if (i < N && !(x(i) == x(i))) kept.clear(i);
        n = 0;
#pragma unroll
        for (int j = 0; j < KeptBits<MAXV>::W; ++j) n += __popcll(kept.w[j]);
    }
    double s = 0.0, m = 0.0, q = 0.0, dmax = 0.0;
    bool final_known = false;
    for (int32_t it = 0; it < max_iters; ++it) {
        if (it == 0 && !MISS)
            clip_pass<MAXV, true, FENCE>(x, kept, N, n, s, m, q, dmax);
        else
            clip_pass<MAXV, false, FENCE>(x, kept, N, n, s, m, q, dmax);
        const double thr = __dmul_rn(ksigma, sqrt(q / (double)n));
        if (!(dmax > thr)) {
            final_known = true;  // nothing drops: m is the mean of the final set
            break;
        }
        int drop = 0;
        clip_fence<FENCE>();
#pragma unroll
        for (int i = 0; i < MAXV; ++i)
            if (kept.get(i) && fabs(__dsub_rn((double)x(i), m)) > thr) {
                kept.clear(i);
                ++drop;
            }
        n -= drop;
        dropped += (unsigned)drop;
    }
    if (final_known) return (float)m;  // m = s / n of this final set
    s = 0.0;
    clip_fence<FENCE>();
#pragma unroll
    for (int i = 0; i < MAXV; ++i)
        if (kept.get(i)) s = __dadd_rn(s, (double)x(i));
    return (float)(s / (double)n);
}

// The column in registers.  Each read goes through an empty asm statement that marks the
// value as changed, so every pass converts it to double again instead of holding the
// column's converted values across the passes (twice the registers; with them a compute
// unit holds fewer waves and the kernel ran 10% slower).
template <int MAXV, bool MISS = false>
__device__ __forceinline__ float clip_registers(const float (&x)[MAXV], int32_t N, double ksigma, int32_t max_iters,
                                                KeptBits<MAXV> &kept, unsigned &dropped)
{
    return clip_values<MAXV, false, MISS>(
        [&](int i) {
            float v = x[i];
            asm volatile("" : "+v"(v));
            return v;
        },
        N, ksigma, max_iters, kept, dropped);
}

// The first iteration of clip_registers alone: true, with the mean, when the column
// settles there (nothing drops, or no iterations are asked for), the same operations in
// the same order as clip_registers, so the mean has the same bits.
template <int MAXV, bool MISS = false>
__device__ __forceinline__ bool clip_first(const float (&x)[MAXV], int32_t N, double ksigma, int32_t max_iters,
                                           float &mean)
{
    auto xv = [&](int i) {
        float v = x[i];
        asm volatile("" : "+v"(v));
        return v;
    };
    KeptBits<MAXV> kept;
    kept.first(N);
    int n = N;
    if (MISS) {
#pragma unroll
        for (int i = 0; i < MAXV; ++i)
            if (i < N && !(x[i] == x[i])) kept.clear(i);
        n = 0;
#pragma unroll
        for (int j = 0; j < KeptBits<MAXV>::W; ++j) n += __popcll(kept.w[j]);
    }
    double s, m, q, dmax;
    if (MISS)
        clip_pass<MAXV, false, false>(xv, kept, N, n, s, m, q, dmax);
    else
        clip_pass<MAXV, true, false>(xv, kept, N, n, s, m, q, dmax);
    if (max_iters > 0 && dmax > __dmul_rn(ksigma, sqrt(q / (double)n))) return false;
    mean = (float)m;
    return true;
}

// PX adjacent pixel columns per thread: each frame's PX values come in as one vector
// load (frame k's plane starts at aligned + k * pstride; pstride >= plane, and pstride
// and the pointers aligned to PX floats; with PX = 4 an even pstride is enough, a frame
// that starts 8-byte aligned taking two 8-byte loads).  Each thread runs the first
// iteration of its columns; a column that drops values there (a few percent of them, but
// in most waves at least one lane) goes to a queue in LDS, and once the workgroup's first
// iterations are done its threads take the queued columns one each (their values kept in
// LDS for columns of up to 32 values and the first 128 queued, else loaded again) and run
// the whole clip, so the later iterations run on full waves instead of holding every wave
// that has one such lane.
// Every result is that of clip_registers on the column.  Columns at or past `plane` are
// neither written nor counted.  The whole workgroup must call this (it synchronises).
template <int MAXV, int PX, bool MISS = false>
__device__ __forceinline__ unsigned combine_cols_block(const float *__restrict__ aligned, int64_t plane,
                                                       int64_t pstride, int32_t N, double ksigma, int32_t max_iters,
                                                       float *__restrict__ out, uint8_t *__restrict__ keep,
                                                       int64_t block)
{
    // queued columns whose values wait in LDS (later ones are loaded again); none for the
    // 48-value columns, whose values held until the queue is written cost more registers
    // than the loads (45 frames of 4096x2048: 0.71 ms loading, 2.05 ms holding them)
    constexpr int QCAP = MAXV <= 32 ? 128 : 0;
    __shared__ int32_t queue[COMB_TILE * PX];         // columns (of this workgroup) that drop values
    __shared__ float qv[MAXV * (QCAP > 0 ? QCAP : 1)];  // value i of queue entry e at qv[i * QCAP + e]
    __shared__ int32_t queued;
    if (threadIdx.x == 0) queued = 0;
    const int64_t p0 = (block * COMB_TILE + threadIdx.x) * PX;
    float xs[PX][MAXV];
    if (PX == 1 || p0 + PX <= plane) {
#pragma unroll
        for (int i = 0; i < MAXV; ++i) {
            if (i < N) {
                const float *src = aligned + (int64_t)i * pstride + p0;
                if (PX == 4 && (((int64_t)i * pstride) & 3) == 0) {
                    const float4 v = *reinterpret_cast<const float4 *>(src);
                    xs[0][i] = v.x;
                    xs[1][i] = v.y;
                    xs[2][i] = v.z;
                    xs[3][i] = v.w;
                } else if (PX == 4) {  // a plane of even length: this frame starts 8-byte aligned
                    const float2 u = *reinterpret_cast<const float2 *>(src);
                    const float2 v = *reinterpret_cast<const float2 *>(src + 2);
                    xs[0][i] = u.x;
                    xs[1][i] = u.y;
                    xs[2][i] = v.x;
                    xs[3][i] = v.y;
                } else if (PX == 2) {
                    const float2 v = *reinterpret_cast<const float2 *>(src);
                    xs[0][i] = v.x;
                    xs[1][i] = v.y;
                } else {
                    xs[0][i] = p0 < plane ? src[0] : 0.0f;
                }
            } else {
#pragma unroll
                for (int c = 0; c < PX; ++c) xs[c][i] = 0.0f;
            }
        }
    } else {
#pragma unroll
        for (int i = 0; i < MAXV; ++i)
#pragma unroll
            for (int c = 0; c < PX; ++c)
                xs[c][i] = (i < N && p0 + c < plane) ? aligned[(int64_t)i * pstride + p0 + c] : 0.0f;
    }
    // first iterations; a column that drops values goes to the workgroup's queue
    float res[PX];
    bool done[PX];
    bool all = p0 + PX <= plane;
#pragma unroll
    for (int c = 0; c < PX; ++c) {
        done[c] = clip_first<MAXV, MISS>(xs[c], N, ksigma, max_iters, res[c]);
        all = all && done[c];
    }
    __syncthreads();  // the queue is empty
    if (PX > 1 && all) {
        if (PX == 4)
            *reinterpret_cast<float4 *>(out + p0) = make_float4(res[0], res[1], res[2], res[3]);
        else
            *reinterpret_cast<float2 *>(out + p0) = make_float2(res[0], res[1]);
    } else {
#pragma unroll
        for (int c = 0; c < PX; ++c)
            if (p0 + c < plane) {
                if (done[c]) {
                    out[p0 + c] = res[c];
                } else {
                    const int32_t e = atomicAdd(&queued, 1);
                    queue[e] = (int32_t)threadIdx.x * PX + c;
                    if (e < QCAP) {
#pragma unroll
                        for (int i = 0; i < MAXV; ++i) qv[i * QCAP + e] = xs[c][i];
                    }
                }
            }
    }
    if (keep) {  // a settled column keeps every value (every value present)
#pragma unroll
        for (int i = 0; i < MAXV; ++i)
            if (i < N)
#pragma unroll
                for (int c = 0; c < PX; ++c)
                    if (p0 + c < plane && done[c])
                        keep[(int64_t)i * plane + p0 + c] = (uint8_t)(!MISS || xs[c][i] == xs[c][i]);
    }
    __syncthreads();
    // the queued columns, one per thread: the whole clip (values from LDS, past QCAP
    // entries loaded again)
    unsigned dropped = 0;
    const int32_t nq = queued;
    for (int32_t e = threadIdx.x; e < nq; e += COMB_TILE) {
        const int64_t p = block * COMB_TILE * PX + queue[e];
        float x[MAXV];
        if (e < QCAP) {
#pragma unroll
            for (int i = 0; i < MAXV; ++i) x[i] = qv[i * QCAP + e];
        } else {
#pragma unroll
            for (int i = 0; i < MAXV; ++i) x[i] = i < N ? aligned[(int64_t)i * pstride + p] : 0.0f;
        }
        KeptBits<MAXV> kept;
        out[p] = clip_registers<MAXV, MISS>(x, N, ksigma, max_iters, kept, dropped);
        if (keep) {
#pragma unroll
            for (int i = 0; i < MAXV; ++i)
                if (i < N) keep[(int64_t)i * plane + p] = (uint8_t)kept.get(i);
        }
    }
    return dropped;
}

// Stacks deeper than a register column: a 64-thread workgroup, one thread per pixel
// column; the first 32 values of a column stay in registers, the others wait in the
// thread's own slice of an LDS tile [N - 32][64] (each thread writes and reads only its
// own column, so no barrier is needed).  The frames
// come in batches of 32 loads in flight; the passes loop over the frames at run time
// with the kept flags in two 64-bit words.  Same arithmetic, in the same order, as
// clip_values (sums over the kept values in frame order, m = s / n, the squared
// deviations and the largest one, the threshold, the drops).  With MISS, NaN values are
// missing: never kept, not counted as dropped, and n counts the others (a pixel with
// none gives NaN).
constexpr int COMB_DEEP_PX = 64;
constexpr int COMB_DEEP_BATCH = 64;  // the most loads a wave keeps in flight
constexpr int COMB_DEEP_REG = 32;    // the first values of a column stay in registers
static_assert(COMB_DEEP_REG < COMB_MAX_N + 1, "the LDS-column kernels serve stacks deeper than COMB_MAX_N");

// f(i, x_i, kept_i) for the values of a column in frame order (f selects rather than
// branches on kept_i): values 0 .. COMB_DEEP_REG-1 from xr, the others from the LDS
// slice col (value i at col[(i - COMB_DEEP_REG) * COMB_DEEP_PX]); the kept flags are
// bit i of k0 (i < 64) and bit i - 64 of k1.  N > COMB_DEEP_REG.
template <typename F>
__device__ __forceinline__ void deep_each(const float (&xr)[COMB_DEEP_REG], const float *col, uint64_t k0,
                                          uint64_t k1, int32_t N, F f)
{
#pragma unroll
    for (int i = 0; i < COMB_DEEP_REG; ++i) f(i, (double)xr[i], ((k0 >> i) & 1ull) != 0);
    uint64_t w = k0 >> COMB_DEEP_REG;
    const int32_t n0 = min(N, 64);
#pragma unroll 4
    for (int i = COMB_DEEP_REG; i < n0; ++i, w >>= 1)
        f(i, (double)col[(i - COMB_DEEP_REG) * COMB_DEEP_PX], (w & 1ull) != 0);
    w = k1;
#pragma unroll 4
    for (int i = 64; i < N; ++i, w >>= 1) f(i, (double)col[(i - COMB_DEEP_REG) * COMB_DEEP_PX], (w & 1ull) != 0);
}

// f(x_i) for every value of a column in frame order (all of them kept: the first
// iteration without missing values).  The empty asm statements mark the register
// values as changed, so each pass converts them to double again instead of holding 32
// converted values (64 more registers) across the passes.
template <typename F>
__device__ __forceinline__ void deep_each_all(float (&xr)[COMB_DEEP_REG], const float *col, int32_t N, F f)
{
#pragma unroll
    for (int i = 0; i < COMB_DEEP_REG; ++i) asm volatile("" : "+v"(xr[i]));
#pragma unroll
    for (int i = 0; i < COMB_DEEP_REG; ++i) f((double)xr[i]);
#pragma unroll 4
    for (int i = COMB_DEEP_REG; i < N; ++i) f((double)col[(i - COMB_DEEP_REG) * COMB_DEEP_PX]);
}

template <bool MISS>
__device__ __forceinline__ unsigned combine_deep_block(const float *__restrict__ aligned, int64_t plane,
                                                       int64_t pstride, int32_t N, double ksigma, int32_t max_iters,
                                                       float *__restrict__ out, uint8_t *__restrict__ keep,
                                                       int64_t block, float *tile)
{
    const int t = threadIdx.x;
    const int64_t p = block * COMB_DEEP_PX + t;
    const float *src = aligned + (p < plane ? p : plane - 1);
    float *col = tile + t;  // values COMB_DEEP_REG .. N-1 (the tile is [N - COMB_DEEP_REG][64])
    float xr[COMB_DEEP_REG];
    for (int32_t i0 = 0; i0 < N; i0 += COMB_DEEP_BATCH) {
        float v[COMB_DEEP_BATCH];
#pragma unroll
        for (int j = 0; j < COMB_DEEP_BATCH; ++j) v[j] = src[(int64_t)min(i0 + j, N - 1) * pstride];
        if (i0 == 0) {
#pragma unroll
            for (int j = 0; j < COMB_DEEP_REG; ++j) xr[j] = v[j];
        }
#pragma unroll
        for (int j = 0; j < COMB_DEEP_BATCH; ++j)
            if (i0 + j >= COMB_DEEP_REG && i0 + j < N) col[(i0 + j - COMB_DEEP_REG) * COMB_DEEP_PX] = v[j];
    }
    uint64_t k0 = N >= 64 ? ~0ull : ((1ull << N) - 1ull);
    uint64_t k1 = N >= 128 ? ~0ull : N <= 64 ? 0ull : ((1ull << (N - 64)) - 1ull);
    int n = N;
    if (MISS) {
        uint64_t m0 = 0, m1 = 0;
        deep_each(xr, col, k0, k1, N, [&](int i, double x, bool k) {
            const uint64_t bit = (k && x == x) ? 1ull : 0ull;
            if (i < 64) m0 |= bit << i;
            else m1 |= bit << (i - 64);
        });
        k0 = m0;
        k1 = m1;
        n = __popcll(k0) + __popcll(k1);
    }
    unsigned dropped = 0;
    // the drop pass of one iteration also forms the next sum (the same values in the
    // same order as a separate pass over the kept set)
    // before the first drop (and without missing values) every value is kept: the same
    // sums without the flag selects
    double s = 0.0;
    if (MISS)
        deep_each(xr, col, k0, k1, N, [&](int, double x, bool k) { s = k ? __dadd_rn(s, x) : s; });
    else
        deep_each_all(xr, col, N, [&](double x) { s = __dadd_rn(s, x); });
    double mean = -1.0;
    bool final_known = false;
    for (int32_t it = 0; it < max_iters; ++it) {
        const double m = s / (double)n;
        double q = 0.0, dmax = 0.0;
        if (!MISS && it == 0)
            deep_each_all(xr, col, N, [&](double x) {
                const double d = __dsub_rn(x, m);
                q = __dadd_rn(q, __dmul_rn(d, d));
                dmax = fmax(dmax, fabs(d));
            });
        else
            deep_each(xr, col, k0, k1, N, [&](int, double x, bool k) {
                const double d = __dsub_rn(x, m);
                q = k ? __dadd_rn(q, __dmul_rn(d, d)) : q;
                dmax = k ? fmax(dmax, fabs(d)) : dmax;
            });
        const double thr = __dmul_rn(ksigma, sqrt(q / (double)n));
        if (!(dmax > thr)) {  // nothing drops: m is the mean of the final set
            mean = m;
            final_known = true;
            break;
        }
        int drop = 0;
        s = 0.0;
        uint64_t n0 = 0, n1 = 0;  // the flags after this iteration
        deep_each(xr, col, k0, k1, N, [&](int i, double x, bool k) {
            const bool out = k && fabs(__dsub_rn(x, m)) > thr;
            const bool stay = k && !out;
            drop += out ? 1 : 0;
            s = stay ? __dadd_rn(s, x) : s;
            const uint64_t bit = stay ? 1ull : 0ull;
            if (i < 64) n0 |= bit << i;
            else n1 |= bit << (i - 64);
        });
        k0 = n0;
        k1 = n1;
        n -= drop;
        dropped += (unsigned)drop;
    }
    if (p >= plane) return 0u;
    out[p] = (float)(final_known ? mean : s / (double)n);
    if (keep)
        for (int i = 0; i < N; ++i)
            keep[(int64_t)i * plane + p] = (uint8_t)((((i < 64 ? k0 : k1) >> (i & 63)) & 1ull) != 0);
    return dropped;
}

}  // namespace rd
