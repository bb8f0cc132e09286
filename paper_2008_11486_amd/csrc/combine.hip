// Sigma-clipped mean co-add along the frame axis (Sections 2.1, 3.1.2).
//
// With one lane per pixel column (the default) each thread loads its column into
// registers directly.  With L > 1 lanes per column a workgroup stages a 256-pixel
// tile of every frame in LDS (one coalesced 1 KB row per frame), then each lane
// takes the frames l, l+L, l+2L, ... of a column and the group's sums, squared
// deviations and drop counts are combined with wavefront butterfly reductions.
// Mean and sigma are evaluated in double.  Bytes per input pixel: 4 read, plus
// 4/N for the output and 1 per value when the keep mask is requested.
#include <cstdlib>

#include "common.h"
#include "combine_core.h"

namespace rd {

template <int L, int MAXV>
__global__ __launch_bounds__(COMB_TILE) void combine_kernel(
    const float *__restrict__ aligned, int64_t plane, int32_t N, double ksigma, int32_t max_iters,
    float *__restrict__ out, uint8_t *__restrict__ keep, unsigned long long *__restrict__ n_rej)
{
    extern __shared__ float tile[];  // [N][COMB_TILE]
    const int64_t p0 = (int64_t)blockIdx.x * COMB_TILE;
    const int t = threadIdx.x;
    for (int32_t k = 0; k < N; ++k) {
        const int64_t p = p0 + t;
        tile[k * COMB_TILE + t] = p < plane ? aligned[k * plane + p] : 0.0f;
    }
    __syncthreads();
    const unsigned dropped_here = clip_tile<L, MAXV>(tile, p0, plane, N, ksigma, max_iters, out, keep);
    if (n_rej) {
        const unsigned total = block_sum_u32(dropped_here);
        if (t == 0 && total) atomicAdd(n_rej, (unsigned long long)total);
    }
}

// One thread per pixel column, the column's N values in registers straight from
// HBM (coalesced across the workgroup's 256 adjacent pixels).  The arithmetic is
// that of clip_column with one lane: sums in frame order in double, m = s / n,
// q = sum of (x - m)^2, threshold ksigma * sqrt(q / n), drop |x - m| > threshold.
// Two shortcuts leave every result unchanged: the largest |x - m| of the q pass
// decides whether the drop pass is needed at all, and when an iteration drops
// nothing its own sum is the final sum.
template <int MAXV, bool ALL>
__device__ __forceinline__ bool kept_at(uint64_t kept, int i, int32_t N)
{
    return ALL ? i < N : ((kept >> i) & 1ull) != 0;
}

template <int MAXV, bool ALL>
__device__ __forceinline__ void clip_pass(const float (&x)[MAXV], uint64_t kept, int32_t N, int n, double &s,
                                          double &m, double &q, double &dmax)
{
    s = 0.0;
#pragma unroll
    for (int i = 0; i < MAXV; ++i)
        if (kept_at<MAXV, ALL>(kept, i, N)) s = __dadd_rn(s, (double)x[i]);
    m = s / (double)n;
    q = 0.0;
    dmax = 0.0;
#pragma unroll
    for (int i = 0; i < MAXV; ++i)
        if (kept_at<MAXV, ALL>(kept, i, N)) {
            const double d = __dsub_rn((double)x[i], m);
            q = __dadd_rn(q, __dmul_rn(d, d));
            dmax = fmax(dmax, fabs(d));
        }
}

// Clip one column held in registers; returns the mean and updates kept / dropped.
template <int MAXV>
__device__ __forceinline__ float clip_registers(const float (&x)[MAXV], int32_t N, double ksigma, int32_t max_iters,
                                                uint64_t &kept, unsigned &dropped)
{
    kept = N >= 64 ? ~0ull : ((1ull << N) - 1ull);
    int n = N;
    double s = 0.0, m = 0.0, q = 0.0, dmax = 0.0;
    bool final_known = false;
    for (int32_t it = 0; it < max_iters; ++it) {
        if (it == 0)
            clip_pass<MAXV, true>(x, kept, N, n, s, m, q, dmax);
        else
            clip_pass<MAXV, false>(x, kept, N, n, s, m, q, dmax);
        const double thr = __dmul_rn(ksigma, sqrt(q / (double)n));
        if (!(dmax > thr)) {
            final_known = true;  // nothing drops: s is the sum over the final set
            break;
        }
        int drop = 0;
#pragma unroll
        for (int i = 0; i < MAXV; ++i)
            if (((kept >> i) & 1ull) && fabs(__dsub_rn((double)x[i], m)) > thr) {
                kept &= ~(1ull << i);
                ++drop;
            }
        n -= drop;
        dropped += (unsigned)drop;
    }
    if (!final_known) {
        s = 0.0;
#pragma unroll
        for (int i = 0; i < MAXV; ++i)
            if ((kept >> i) & 1ull) s = __dadd_rn(s, (double)x[i]);
    }
    return (float)(s / (double)n);
}

// PX adjacent pixel columns per thread: each frame's PX values come in as one vector
// load (plane and pointer aligned to PX floats), then the columns are clipped one
// after the other.
template <int MAXV, int PX>
__global__ __launch_bounds__(COMB_TILE) void combine_cols(
    const float *__restrict__ aligned, int64_t plane, int32_t N, double ksigma, int32_t max_iters,
    float *__restrict__ out, uint8_t *__restrict__ keep, unsigned long long *__restrict__ n_rej)
{
    const int64_t p0 = ((int64_t)blockIdx.x * COMB_TILE + threadIdx.x) * PX;
    float xs[PX][MAXV];
    if (PX == 1 || p0 + PX <= plane) {
#pragma unroll
        for (int i = 0; i < MAXV; ++i) {
            if (i < N) {
                const float *src = aligned + (int64_t)i * plane + p0;
                if (PX == 4) {
                    const float4 v = *reinterpret_cast<const float4 *>(src);
                    xs[0][i] = v.x;
                    xs[1][i] = v.y;
                    xs[2][i] = v.z;
                    xs[3][i] = v.w;
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
                xs[c][i] = (i < N && p0 + c < plane) ? aligned[(int64_t)i * plane + p0 + c] : 0.0f;
    }
    unsigned dropped = 0;
    float res[PX];
    uint64_t kept[PX];
#pragma unroll
    for (int c = 0; c < PX; ++c) {
        unsigned d = 0;
        res[c] = clip_registers<MAXV>(xs[c], N, ksigma, max_iters, kept[c], d);
        if (p0 + c < plane) dropped += d;
    }
    if (PX > 1 && p0 + PX <= plane) {
        if (PX == 4)
            *reinterpret_cast<float4 *>(out + p0) = make_float4(res[0], res[1], res[2], res[3]);
        else
            *reinterpret_cast<float2 *>(out + p0) = make_float2(res[0], res[1]);
    } else {
#pragma unroll
        for (int c = 0; c < PX; ++c)
            if (p0 + c < plane) out[p0 + c] = res[c];
    }
    if (keep) {
#pragma unroll
        for (int i = 0; i < MAXV; ++i)
            if (i < N)
#pragma unroll
                for (int c = 0; c < PX; ++c)
                    if (p0 + c < plane) keep[(int64_t)i * plane + p0 + c] = (uint8_t)((kept[c] >> i) & 1ull);
    }
    if (n_rej) {
        const unsigned total = block_sum_u32(dropped);
        if (threadIdx.x == 0 && total) atomicAdd(n_rej, (unsigned long long)total);
    }
}

__global__ void zero_u64(unsigned long long *p) { *p = 0ull; }

// Pixel columns per thread of the one-lane kernel (at most 4); REDUCE_COMBINE_PX overrides.
static int combine_px()
{
    const char *e = std::getenv("REDUCE_COMBINE_PX");
    if (e) {
        const int v = std::atoi(e);
        if (v == 1 || v == 2 || v == 4) return v;
    }
    return 4;
}

void combine_dispatch(int lanes, const float *aligned, int64_t plane, int32_t N, double ksigma, int32_t max_iters,
                      float *out, uint8_t *keep, unsigned long long *n_rej, hipStream_t s)
{
    const unsigned blocks = (unsigned)ceil_div(plane, COMB_TILE);
    const size_t lds = sizeof(float) * (size_t)N * COMB_TILE;
    ProfScope prof("combine", s);
    auto launch = [&](auto Lc, auto Vc) {
        constexpr int L = decltype(Lc)::value, V = decltype(Vc)::value;
        hipLaunchKernelGGL((combine_kernel<L, V>), dim3(blocks), dim3(COMB_TILE), lds, s, aligned, plane, N, ksigma,
                           max_iters, out, keep, n_rej);
    };
    // vector loads need the frame planes and the pointer aligned to the pixel group
    const bool v4 = plane % 4 == 0 && (reinterpret_cast<uintptr_t>(aligned) & 15u) == 0 &&
                    (reinterpret_cast<uintptr_t>(out) & 15u) == 0;
    const bool v2 = plane % 2 == 0 && (reinterpret_cast<uintptr_t>(aligned) & 7u) == 0 &&
                    (reinterpret_cast<uintptr_t>(out) & 7u) == 0;
    auto launch_cols = [&](auto Vc, auto Pc) {
        constexpr int V = decltype(Vc)::value, P = decltype(Pc)::value;
        hipLaunchKernelGGL((combine_cols<V, P>), dim3((unsigned)ceil_div(plane, (int64_t)COMB_TILE * P)),
                           dim3(COMB_TILE), 0, s, aligned, plane, N, ksigma, max_iters, out, keep, n_rej);
    };
    const int px = combine_px();
    switch (lanes) {
    case 1:
        if (N <= 16) {
            if (v4 && px >= 4) launch_cols(std::integral_constant<int, 16>{}, std::integral_constant<int, 4>{});
            else if (v2 && px >= 2) launch_cols(std::integral_constant<int, 16>{}, std::integral_constant<int, 2>{});
            else launch_cols(std::integral_constant<int, 16>{}, std::integral_constant<int, 1>{});
        } else if (N <= 32) {
            if (v2 && px >= 2) launch_cols(std::integral_constant<int, 32>{}, std::integral_constant<int, 2>{});
            else launch_cols(std::integral_constant<int, 32>{}, std::integral_constant<int, 1>{});
        } else {
            launch_cols(std::integral_constant<int, 48>{}, std::integral_constant<int, 1>{});
        }
        break;
    case 2: launch(std::integral_constant<int, 2>{}, std::integral_constant<int, 24>{}); break;
    case 4: launch(std::integral_constant<int, 4>{}, std::integral_constant<int, 12>{}); break;
    case 8: launch(std::integral_constant<int, 8>{}, std::integral_constant<int, 6>{}); break;
    case 16: launch(std::integral_constant<int, 16>{}, std::integral_constant<int, 3>{}); break;
    case 32: launch(std::integral_constant<int, 32>{}, std::integral_constant<int, 2>{}); break;
    default: launch(std::integral_constant<int, 64>{}, std::integral_constant<int, 1>{}); break;
    }
}

int combine_lanes_for(int32_t N);

}  // namespace rd

using namespace rd;

extern "C" int reduce_combine(const float *aligned, int32_t w, int32_t h, int32_t N, float ksigma,
                              int32_t max_iters, float *out, uint8_t *keep, int64_t *n_rej, void *stream)
{
    if (!aligned || !out) return fail(REDUCE_ERR_NULL, "reduce_combine: NULL buffer");
    if (w < 1 || h < 1 || N < 1) return fail(REDUCE_ERR_SHAPE, "reduce_combine: w, h, N must be >= 1");
    if (!(ksigma > 0.0f) || !std::isfinite(ksigma) || max_iters < 0)
        return fail(REDUCE_ERR_RANGE, "reduce_combine: ksigma must be > 0 and max_iters >= 0");
    if (N > COMB_MAX_N) return fail(REDUCE_ERR_UNSUPPORTED, "reduce_combine: N above 48");
    hipStream_t s = as_stream(stream);
    unsigned long long *nr = reinterpret_cast<unsigned long long *>(n_rej);
    if (nr) hipLaunchKernelGGL(zero_u64, dim3(1), dim3(1), 0, s, nr);
    combine_dispatch(combine_lanes_for(N), aligned, (int64_t)w * h, N, (double)ksigma, max_iters, out, keep, nr, s);
    return check_launch("reduce_combine");
}
