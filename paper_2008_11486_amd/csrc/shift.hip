// Bilinear sub-pixel shift onto the common overlap (Section 3.2.1 names bilinear
// interpolation as the cheaper alternative to the paper's bicubic spline).
//
// Streaming kernel, 4 consecutive outputs of one row per thread.  The integer part
// of the offset is applied in integer arithmetic, the fraction becomes per-frame
// bilinear weights evaluated in double and rounded once.  Bytes per output pixel:
// 4 read (each input row is read by two output rows, served from cache) + 4 write.
#include "common.h"

namespace rd {

constexpr int SH_VEC = 4;
constexpr int SH_BLOCK = 256;

__device__ __forceinline__ int32_t clampi(int32_t v, int32_t lo, int32_t hi)
{
    return v < lo ? lo : (v > hi ? hi : v);
}

template <bool INTEGER>
__global__ __launch_bounds__(SH_BLOCK) void shift_kernel(
    const float *__restrict__ in, float *__restrict__ out, int32_t W, int32_t H,
    const float *__restrict__ offs, int32_t x0, int32_t y0, int32_t w, int32_t h, bool vec_store)
{
    const int32_t k = blockIdx.z;
    const int32_t v = blockIdx.y;
    const int32_t u0 = (blockIdx.x * SH_BLOCK + threadIdx.x) * SH_VEC;
    if (u0 >= w) return;
    const ShiftSetup ss = shift_setup(offs[2 * k], offs[2 * k + 1]);
    const float *f = in + (int64_t)k * W * H;
    float *o = out + ((int64_t)k * h + v) * w;
    const int32_t j = clampi(y0 + v + ss.iy, 0, H - 1);
    float r[SH_VEC];
    if (INTEGER) {
#pragma unroll
        for (int e = 0; e < SH_VEC; ++e) r[e] = f[(int64_t)j * W + clampi(x0 + u0 + e + ss.ix, 0, W - 1)];
    } else {
        const int32_t j1 = clampi(ss.b > 0.0 ? j + 1 : j, 0, H - 1);
        const int32_t step = ss.a > 0.0 ? 1 : 0;
        float t0[SH_VEC + 1], t1[SH_VEC + 1];
#pragma unroll
        for (int e = 0; e <= SH_VEC; ++e) {
            const int32_t i = clampi(x0 + u0 + e + ss.ix, 0, W - 1);
            t0[e] = f[(int64_t)j * W + i];
            t1[e] = f[(int64_t)j1 * W + i];
        }
#pragma unroll
        for (int e = 0; e < SH_VEC; ++e) {
            // the right-hand tap is the next column only when it carries weight
            const float f10 = step ? t0[e + 1] : t0[e];
            const float f11 = step ? t1[e + 1] : t1[e];
            r[e] = bilerp(ss.a, ss.b, t0[e], f10, t1[e], f11);
        }
    }
    if (vec_store && u0 + SH_VEC <= w) {
        *reinterpret_cast<float4 *>(o + u0) = make_float4(r[0], r[1], r[2], r[3]);
    } else {
#pragma unroll
        for (int e = 0; e < SH_VEC; ++e)
            if (u0 + e < w) o[u0 + e] = r[e];
    }
}

}  // namespace rd

using namespace rd;

extern "C" int reduce_shift(const float *in, float *out, int32_t W, int32_t H, int32_t N,
                            const float *offs, const int32_t *rect, int32_t integer_mode, void *stream)
{
    if (!in || !out || !offs || !rect) return fail(REDUCE_ERR_NULL, "reduce_shift: NULL argument");
    if (W < 1 || H < 1 || N < 1) return fail(REDUCE_ERR_SHAPE, "reduce_shift: W, H, N must be >= 1");
    const int32_t x0 = rect[0], y0 = rect[1], w = rect[2], h = rect[3];
    if (w < 1 || h < 1 || w > W || h > H) return fail(REDUCE_ERR_SHAPE, "reduce_shift: empty or oversized rect");
    if (N > 65535 || h > 65535) return fail(REDUCE_ERR_UNSUPPORTED, "reduce_shift: N or h above 65535");
    const bool vec_store = (w % SH_VEC == 0) && ((reinterpret_cast<uintptr_t>(out) & 15u) == 0);
    dim3 grid((unsigned)ceil_div(w, (int64_t)SH_BLOCK * SH_VEC), (unsigned)h, (unsigned)N);
    ProfScope prof("shift", as_stream(stream));
    if (integer_mode)
        hipLaunchKernelGGL(shift_kernel<true>, grid, dim3(SH_BLOCK), 0, as_stream(stream), in, out, W, H, offs, x0,
                           y0, w, h, vec_store);
    else
        hipLaunchKernelGGL(shift_kernel<false>, grid, dim3(SH_BLOCK), 0, as_stream(stream), in, out, W, H, offs, x0,
                           y0, w, h, vec_store);
    return check_launch("reduce_shift");
}
