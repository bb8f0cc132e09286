// Device routine of the sigma-clipped mean over one pixel column held by a group of
// L lanes; used by the stage-wise combine kernel and by the fused batch kernel so
// both evaluate identical operations in identical order.
#pragma once

#include <type_traits>

#include "common.h"

namespace rd {

constexpr int COMB_TILE = 256;
constexpr int COMB_MAX_N = 48;  // LDS tile [N][256] floats stays within 48 KB

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

}  // namespace rd
