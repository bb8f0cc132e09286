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

// PX adjacent pixel columns per thread (combine_cols_block); one atomic per workgroup
// for the rejection count.  MISS: NaN values are missing.
template <int MAXV, int PX, bool MISS>
__global__ __launch_bounds__(COMB_TILE) void combine_cols(
    const float *__restrict__ aligned, int64_t plane, int32_t N, double ksigma, int32_t max_iters,
    float *__restrict__ out, uint8_t *__restrict__ keep, unsigned long long *__restrict__ n_rej)
{
    const unsigned dropped = combine_cols_block<MAXV, PX, MISS>(aligned, plane, plane, N, ksigma, max_iters, out,
                                                                keep, (int64_t)blockIdx.x);
    if (n_rej) {
        const unsigned total = block_sum_u32(dropped);
        if (threadIdx.x == 0 && total) atomicAdd(n_rej, (unsigned long long)total);
    }
}

// Stacks of 49 - 128 frames, and stacks with missing values: 64 pixel columns per
// workgroup, values in LDS [N][64].
template <bool MISS>
__global__ __launch_bounds__(COMB_DEEP_PX) __attribute__((amdgpu_waves_per_eu(3))) void combine_deep(
    const float *__restrict__ aligned, int64_t plane, int32_t N, double ksigma, int32_t max_iters,
    float *__restrict__ out, uint8_t *__restrict__ keep, unsigned long long *__restrict__ n_rej)
{
    extern __shared__ float tile[];
    unsigned dropped = combine_deep_block<MISS>(aligned, plane, plane, N, ksigma, max_iters, out, keep,
                                                (int64_t)blockIdx.x, tile);
    if (n_rej) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) dropped += __shfl_xor(dropped, off, 64);
        if (threadIdx.x == 0 && dropped) atomicAdd(n_rej, (unsigned long long)dropped);
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

static void launch_deep(bool missing, const float *aligned, int64_t plane, int32_t N, double ksigma,
                        int32_t max_iters, float *out, uint8_t *keep, unsigned long long *n_rej, hipStream_t s)
{
    const dim3 grid((unsigned)ceil_div(plane, (int64_t)COMB_DEEP_PX));
    const size_t lds = sizeof(float) * (N - COMB_DEEP_REG) * COMB_DEEP_PX;
    if (missing)
        hipLaunchKernelGGL(combine_deep<true>, grid, dim3(COMB_DEEP_PX), lds, s, aligned, plane, N, ksigma, max_iters,
                           out, keep, n_rej);
    else
        hipLaunchKernelGGL(combine_deep<false>, grid, dim3(COMB_DEEP_PX), lds, s, aligned, plane, N, ksigma,
                           max_iters, out, keep, n_rej);
}

// One lane per column (missing = 1 takes only this path): registers up to 48 frames,
// the LDS-column kernel past that.
template <bool MISS>
static void dispatch_cols(const float *aligned, int64_t plane, int32_t N, double ksigma, int32_t max_iters,
                          float *out, uint8_t *keep, unsigned long long *n_rej, hipStream_t s)
{
    // vector loads need the frame planes and the pointer aligned to the pixel group (four
    // pixels: frames of even length, 8-byte loads where a frame starts off 16 bytes)
    const bool v4 = plane % 2 == 0 && (reinterpret_cast<uintptr_t>(aligned) & 15u) == 0 &&
                    (reinterpret_cast<uintptr_t>(out) & 15u) == 0;
    const bool v2 = plane % 2 == 0 && (reinterpret_cast<uintptr_t>(aligned) & 7u) == 0 &&
                    (reinterpret_cast<uintptr_t>(out) & 7u) == 0;
    auto launch_cols = [&](auto Vc, auto Pc) {
        constexpr int V = decltype(Vc)::value, P = decltype(Pc)::value;
        hipLaunchKernelGGL((combine_cols<V, P, MISS>), dim3((unsigned)ceil_div(plane, (int64_t)COMB_TILE * P)),
                           dim3(COMB_TILE), 0, s, aligned, plane, N, ksigma, max_iters, out, keep, n_rej);
    };
    const int px = combine_px();
    if (N <= 16) {
        if (v4 && px >= 4) launch_cols(std::integral_constant<int, 16>{}, std::integral_constant<int, 4>{});
        else if (v2 && px >= 2) launch_cols(std::integral_constant<int, 16>{}, std::integral_constant<int, 2>{});
        else launch_cols(std::integral_constant<int, 16>{}, std::integral_constant<int, 1>{});
    } else if (N <= 32) {
        if (v2 && px >= 2) launch_cols(std::integral_constant<int, 32>{}, std::integral_constant<int, 2>{});
        else launch_cols(std::integral_constant<int, 32>{}, std::integral_constant<int, 1>{});
    } else if (N <= 48) {
        launch_cols(std::integral_constant<int, 48>{}, std::integral_constant<int, 1>{});
    } else {
        launch_deep(MISS, aligned, plane, N, ksigma, max_iters, out, keep, n_rej, s);
    }
}

void combine_dispatch(int lanes, const float *aligned, int64_t plane, int32_t N, double ksigma, int32_t max_iters,
                      float *out, uint8_t *keep, unsigned long long *n_rej, hipStream_t s)
{
    const unsigned blocks = (unsigned)ceil_div(plane, COMB_TILE);
    const size_t lds = sizeof(float) * (size_t)N * COMB_TILE;
    ProfScope prof(N > COMB_MAX_N ? "combine_deep" : "combine", s);
    auto launch = [&](auto Lc, auto Vc) {
        constexpr int L = decltype(Lc)::value, V = decltype(Vc)::value;
        hipLaunchKernelGGL((combine_kernel<L, V>), dim3(blocks), dim3(COMB_TILE), lds, s, aligned, plane, N, ksigma,
                           max_iters, out, keep, n_rej);
    };
    switch (lanes) {
    case 1: dispatch_cols<false>(aligned, plane, N, ksigma, max_iters, out, keep, n_rej, s); break;
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
                              int32_t max_iters, float *out, uint8_t *keep, int64_t *n_rej, int32_t missing,
                              void *stream)
{
    if (!aligned || !out) return fail(REDUCE_ERR_NULL, "reduce_combine: NULL buffer");
    if (w < 1 || h < 1 || N < 1) return fail(REDUCE_ERR_SHAPE, "reduce_combine: w, h, N must be >= 1");
    if (!(ksigma > 0.0f) || !std::isfinite(ksigma) || max_iters < 0)
        return fail(REDUCE_ERR_RANGE, "reduce_combine: ksigma must be > 0 and max_iters >= 0");
    if (N > COMB_MAX_N_COLS) return fail(REDUCE_ERR_UNSUPPORTED, "reduce_combine: N above 128");
    hipStream_t s = as_stream(stream);
    unsigned long long *nr = reinterpret_cast<unsigned long long *>(n_rej);
    if (nr) hipLaunchKernelGGL(zero_u64, dim3(1), dim3(1), 0, s, nr);
    if (missing) {
        // values that are NaN (bad pixels) are left out: one lane per column
        ProfScope prof("combine_missing", s);
        dispatch_cols<true>(aligned, (int64_t)w * h, N, (double)ksigma, max_iters, out, keep, nr, s);
        return check_launch("reduce_combine");
    }
    // past the LDS tile's depth only the one-lane kernel (column in registers) applies
    const int lanes = N > COMB_MAX_N ? 1 : combine_lanes_for(N);
    combine_dispatch(lanes, aligned, (int64_t)w * h, N, (double)ksigma, max_iters, out, keep, nr, s);
    return check_launch("reduce_combine");
}
