// Star-field renderer for the offset-proposal network's training and evaluation
// pairs, and the conversion of the network's prediction into search-window centres.
//
// A frame is sky + circular Gaussian stars + Gaussian noise whose variance is the
// signal plus the read-noise variance (the normal approximation of photon noise at
// sky levels of ~1000 e-).  Star catalogues come from the caller; the noise comes
// from a counter-based generator keyed by (seed, frame key, pixel), so a frame is a
// pure function of its inputs and re-rendering gives the same pixels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>

#include "common.h"

namespace rd {

constexpr int RT_X = 64, RT_Y = 64;   // pixels per render tile
constexpr int RT_STAMP = 8;           // a star reaches pixels within +-8 px of its centre

// Philox4x32 with 10 rounds (Salmon, Moraes, Dror and Shaw, "Parallel random numbers:
// as easy as 1, 2, 3", SC 2011): each round multiplies two counter words by fixed
// odd constants, mixes the high and low halves with the other words and the key,
// and the key is bumped by the Weyl constants between rounds.
struct U4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c = U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// one standard normal from two 32-bit words (Box-Muller, cosine branch)
__device__ __forceinline__ float std_normal(uint32_t a, uint32_t b)
{
    const float u1 = ((float)a + 1.0f) * 2.3283064365386963e-10f;  // (0, 1]
    const float u2 = (float)b * 2.3283064365386963e-10f;           // [0, 1)
    return sqrtf(-2.0f * logf(u1)) * cosf(6.283185307179586f * u2);
}

// Grid (tiles_x, tiles_y, F).  The workgroup walks the frame's catalogue in chunks
// of 256 stars, keeps (in catalogue order) those within the stamp reach of its tile,
// and every thread adds them to its 16 pixels, so the sum order is fixed.
__global__ __launch_bounds__(256) void render_kernel(const float4 *__restrict__ stars, int32_t S,
                                                     const int64_t *__restrict__ keys, int32_t W, int32_t H,
                                                     float sky, float inv2s2, float read_var, int32_t noise,
                                                     uint32_t seed_lo, uint32_t seed_hi, float *__restrict__ out)
{
    __shared__ float4 list[256];
    __shared__ int32_t wave_cnt[4];
    const int32_t f = blockIdx.z;
    const int32_t x0 = blockIdx.x * RT_X, y0 = blockIdx.y * RT_Y;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    float acc[RT_Y / 4];
#pragma unroll
    for (int i = 0; i < RT_Y / 4; ++i) acc[i] = 0.0f;
    const float4 *cat = stars + (int64_t)f * S;
    const float lo_x = x0 - RT_STAMP - 0.5f, hi_x = x0 + RT_X + RT_STAMP - 0.5f;
    const float lo_y = y0 - RT_STAMP - 0.5f, hi_y = y0 + RT_Y + RT_STAMP - 0.5f;

    for (int32_t base = 0; base < S; base += 256) {
        const int32_t i = base + threadIdx.x;
        float4 st = make_float4(0.f, 0.f, 0.f, 0.f);
        bool keep = false;
        if (i < S) {
            st = cat[i];
            keep = st.x >= lo_x && st.x <= hi_x && st.y >= lo_y && st.y <= hi_y;
        }
        const uint64_t mask = __ballot(keep);
        const int32_t before = __popcll(mask & ((1ull << lane) - 1ull));
        if (lane == 0) wave_cnt[wave] = __popcll(mask);
        __syncthreads();
        int32_t off = 0, n = 0;
        for (int w = 0; w < 4; ++w) {
            if (w < wave) off += wave_cnt[w];
            n += wave_cnt[w];
        }
        if (keep) list[off + before] = st;
        __syncthreads();
        const float px = (float)(x0 + tx);
        for (int32_t j = 0; j < n; ++j) {
            const float4 s = list[j];
            const float dx = px - s.x;
            if (fabsf(dx) > (float)RT_STAMP) continue;
#pragma unroll
            for (int r = 0; r < RT_Y / 4; ++r) {
                const float dy = (float)(y0 + ty + 4 * r) - s.y;
                if (fabsf(dy) <= (float)RT_STAMP) acc[r] += s.z * expf(-(dx * dx + dy * dy) * inv2s2);
            }
        }
        __syncthreads();
    }
    const uint64_t key = (uint64_t)keys[f];
    const int32_t x = x0 + tx;
    if (x >= W) return;
#pragma unroll
    for (int r = 0; r < RT_Y / 4; ++r) {
        const int32_t y = y0 + ty + 4 * r;
        if (y >= H) continue;
        const float sig = sky + acc[r];
        if (!noise) {
            out[((int64_t)f * H + y) * W + x] = sig;
            continue;
        }
        const uint64_t pix = (uint64_t)y * (uint64_t)W + (uint64_t)x;
        const U4 rnd = philox4x32_10(U4{(uint32_t)pix, (uint32_t)(pix >> 32), (uint32_t)key, (uint32_t)(key >> 32)},
                                     seed_lo, seed_hi);
        const float v = sig + sqrtf(fmaxf(sig, 0.0f) + read_var) * std_normal(rnd.x, rnd.y);
        out[((int64_t)f * H + y) * W + x] = v;
    }
}

__global__ void centres_kernel(const float *__restrict__ pred, int32_t B, float scale, int32_t rmax,
                               int32_t *__restrict__ centres)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 2 * B) return;
    const float v = rintf(scale * pred[i]);
    const float c = fminf(fmaxf(v, (float)-rmax), (float)rmax);  // NaN becomes -rmax
    centres[i] = (int32_t)c;
}

// A window whose maximum sits on a border inside the search limit moves its centre
// onto that maximum (a border at +-rmax is also the full search's border).
__global__ void recentre_kernel(const reduce_offset_t *__restrict__ offs, int32_t N, int32_t rmax,
                                int32_t *__restrict__ centres)
{
    const int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    const reduce_offset_t o = offs[k];
    const bool bx = (o.flags & REDUCE_EDGE_X) && o.dx > -rmax && o.dx < rmax;
    const bool by = (o.flags & REDUCE_EDGE_Y) && o.dy > -rmax && o.dy < rmax;
    if (bx || by) {
        centres[2 * k] = min(max(o.dx, -rmax), rmax);
        centres[2 * k + 1] = min(max(o.dy, -rmax), rmax);
    }
}

}  // namespace rd

using namespace rd;

extern "C" int reduce_render_frames(const float *stars, int32_t S, const int64_t *keys, int32_t F, int32_t W,
                                    int32_t H, float sky, float fwhm, float read_noise, int32_t noise, uint64_t seed,
                                    float *out, void *stream)
{
    if ((!stars && S > 0) || !keys || !out) return fail(REDUCE_ERR_NULL, "reduce_render_frames: NULL buffer");
    if (S < 0 || F < 1 || W < 1 || H < 1) return fail(REDUCE_ERR_SHAPE, "reduce_render_frames: bad sizes");
    if (F > 65535) return fail(REDUCE_ERR_UNSUPPORTED, "reduce_render_frames: F above 65535");
    if (!(fwhm > 0.0f) || !(sky >= 0.0f) || !(read_noise >= 0.0f))
        return fail(REDUCE_ERR_RANGE, "reduce_render_frames: fwhm > 0, sky >= 0, read_noise >= 0 needed");
    const double sigma = (double)fwhm / (2.0 * std::sqrt(2.0 * std::log(2.0)));
    const float inv2s2 = (float)(1.0 / (2.0 * sigma * sigma));
    dim3 grid((unsigned)ceil_div(W, RT_X), (unsigned)ceil_div(H, RT_Y), (unsigned)F);
    ProfScope prof("render", as_stream(stream));
    hipLaunchKernelGGL(render_kernel, grid, dim3(256), 0, as_stream(stream), reinterpret_cast<const float4 *>(stars),
                       S, keys, W, H, sky, inv2s2, read_noise * read_noise, noise, (uint32_t)seed, (uint32_t)(seed >> 32),
                       out);
    return check_launch("reduce_render_frames");
}

extern "C" int reduce_cnn_centres(const float *pred, int32_t B, float scale, int32_t radius_max, int32_t *centres,
                                  void *stream)
{
    if (!pred || !centres) return fail(REDUCE_ERR_NULL, "reduce_cnn_centres: NULL buffer");
    if (B < 1) return fail(REDUCE_ERR_SHAPE, "reduce_cnn_centres: B must be >= 1");
    if (radius_max < 0 || !std::isfinite(scale)) return fail(REDUCE_ERR_RANGE, "reduce_cnn_centres: bad range");
    hipLaunchKernelGGL(centres_kernel, dim3((unsigned)ceil_div(2 * (int64_t)B, 256)), dim3(256), 0,
                       as_stream(stream), pred, B, scale, radius_max, centres);
    return check_launch("reduce_cnn_centres");
}

extern "C" int reduce_recentre(const reduce_offset_t *offs, int32_t N, int32_t radius_max, int32_t *centres,
                               void *stream)
{
    if (!offs || !centres) return fail(REDUCE_ERR_NULL, "reduce_recentre: NULL buffer");
    if (N < 1) return fail(REDUCE_ERR_SHAPE, "reduce_recentre: N must be >= 1");
    if (radius_max < 0) return fail(REDUCE_ERR_RANGE, "reduce_recentre: negative radius_max");
    hipLaunchKernelGGL(recentre_kernel, dim3((unsigned)ceil_div(N, 256)), dim3(256), 0, as_stream(stream), offs, N,
                       radius_max, centres);
    return check_launch("reduce_recentre");
}
