// Device routine of the sigma-clipped mean over one pixel column held by a group of
// L lanes; used by the stage-wise combine kernel and by the fused batch kernel so
// both evaluate identical operations in identical order.
#pragma once

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
// or after max_iters passes, return the mean of what is kept.  With L = 1 the sums
// run over the frames in index order.
template <int L, int MAXV>
__device__ __forceinline__ ClipResult<MAXV> clip_column(const float (&x)[MAXV], int32_t N, int lane, double ksigma,
                                                        int32_t max_iters)
{
    uint64_t kept = 0;
#pragma unroll
    for (int i = 0; i < MAXV; ++i)
        if (lane + L * i < N) kept |= (1ull << i);
    int n = N;
    int dropped = 0;
    for (int32_t it = 0; it < max_iters; ++it) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < MAXV; ++i)
            if ((kept >> i) & 1ull) s = __dadd_rn(s, (double)x[i]);
        s = group_sum<L>(s);
        const double m = s / (double)n;
        double q = 0.0;
#pragma unroll
        for (int i = 0; i < MAXV; ++i)
            if ((kept >> i) & 1ull) {
                const double d = __dsub_rn((double)x[i], m);
                q = __dadd_rn(q, __dmul_rn(d, d));
            }
        q = group_sum<L>(q);
        const double thr = __dmul_rn(ksigma, sqrt(q / (double)n));
        int drop = 0;
#pragma unroll
        for (int i = 0; i < MAXV; ++i)
            if (((kept >> i) & 1ull) && fabs(__dsub_rn((double)x[i], m)) > thr) {
                kept &= ~(1ull << i);
                ++drop;
            }
        drop = group_sum<L>(drop);
        n -= drop;
        dropped += drop;
        if (drop == 0) break;
    }
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < MAXV; ++i)
        if ((kept >> i) & 1ull) s = __dadd_rn(s, (double)x[i]);
    s = group_sum<L>(s);
    ClipResult<MAXV> r;
    r.mean = (float)(s / (double)n);
    r.kept = kept;
    r.dropped = dropped;
    return r;
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
